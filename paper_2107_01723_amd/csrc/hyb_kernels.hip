// HIP kernels of the hybrid-PIC step for gfx950 (CDNA4, 64-wide waves).
//
// Every kernel is "batched": it receives the device array of run
// descriptors and a block map that assigns each workgroup to one run and a
// block index inside that run, so one launch serves a single run or many
// resident runs of the serving engine.  All loops are grid-stride over
// counts read from device memory, so a step can be captured once as a HIP
// graph and replayed while particles are injected and removed.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "hyb_internal.h"
#include "hyb_kernels.h"
#include "hyb_solid.h"

namespace hyb {

constexpr int kBlock = kChunk;
constexpr int kWaves = kBlock / 64;
constexpr int kHalo = kTile + 2;              // node span of a tile's stencils
constexpr int kHaloN = kHalo * kHalo * kHalo; // 216

// integer adds into LDS words
__device__ __forceinline__ void lds_add(long long* p, long long v) {
  atomicAdd((unsigned long long*)p, (unsigned long long)v);
}
__device__ __forceinline__ void lds_add(int* p, int v) { atomicAdd(p, v); }

// Number of electrons sources inject at `step`, and per-source first id.
__device__ __forceinline__ long long inject_count(const RunDesc& R, long long step,
                                                  long long* cnt = nullptr, long long* first = nullptr) {
  long long tot = 0;
  for (int s = 0; s < R.nsrc; ++s) {
    const gptr<const SourceDesc> S = G(R.src) + s;
    const long long i = step - S->s0;
    long long c = 0;
    if (i >= 0 && i < S->ns) c = S->base + (i < S->rem ? 1 : 0);
    if (cnt) cnt[s] = c;
    if (first) first[s] = S->id0 + i * S->base + (i < S->rem ? i : S->rem);
    tot += c;
  }
  return tot;
}

// Number of electrons the sources will inject after `step`: the particle
// slots that delta rays must leave free.
__device__ __forceinline__ long long later_injections(const RunDesc& R, long long step) {
  long long tot = 0;
  for (int s = 0; s < R.nsrc; ++s) {
    const gptr<const SourceDesc> S = G(R.src) + s;
    long long i0 = step + 1 - S->s0;
    i0 = i0 > 0 ? i0 : 0;
    if (i0 >= S->ns) continue;
    const long long extra = (S->rem < S->ns ? S->rem : S->ns) - i0;
    tot += (S->ns - i0) * S->base + (extra > 0 ? extra : 0);
  }
  return tot;
}

// Block-wide sum of per-thread integer accumulators, then one atomic per
// non-zero term: ledger terms to `led`, event counts to `evt`.  The
// registers hold the NL ledger terms and the first NC event counts; `extra`,
// if given, holds block-wide LDS sums of all NT terms in the same order.
template <int NL, int NC, int NT = NL + NC>
__device__ __forceinline__ void block_flush(const long long (&v)[NL + NC], long long* __restrict__ led,
                                            long long* __restrict__ evt, const long long* extra = nullptr) {
  __shared__ long long sm[kWaves][NL + NC];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NL + NC; ++i) {
    long long x = v[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0) sm[wave][i] = x;
  }
  __syncthreads();
  if (threadIdx.x < NT) {
    long long s = 0;
    if (threadIdx.x < NL + NC)
#pragma unroll
      for (int w = 0; w < kWaves; ++w) s += sm[w][threadIdx.x];
    if (extra) s += extra[threadIdx.x];
    if (s != 0) {
      long long* dst = threadIdx.x < NL ? &led[threadIdx.x] : &evt[threadIdx.x - NL];
      atomic_add_i64(dst, s);
    }
  }
}

// Cell index and offset of a coordinate (cell units), kept inside [0, n).
template <typename T>
__device__ __forceinline__ void to_cell(T x, int n, int& c, T& o) {
  T f = m_floor(x);
  if (!(f >= (T)0)) { c = 0; o = (T)0; return; }
  if (f > (T)(n - 1)) { c = n - 1; o = (T)1 - (T)(sizeof(T) == 4 ? 5.9604644775390625e-08 : 1.1102230246251565e-16); return; }
  c = (int)f;
  o = x - f;
}

// ---------------------------------------------------------------------------
// injection (App. B exponential spectrum; Sec. II.B spot and cone)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_inject(const RunDesc* __restrict__ runs,
                                                   const BlockMap* __restrict__ bmap) {
  const BlockMap bm = bmap[blockIdx.x];
  const RunDesc& R = runs[bm.run];
  const auto ctr = G(R.ctr);
  if (!ctr->active) return;
  const long long step = ctr->step;
  const long long n0 = ctr->n_total;
  const PartG<T> P = part_g<T>(R.p[ctr->cur]);
  long long cnt[kMaxSources], first[kMaxSources];
  const long long tot = inject_count(R, step, cnt, first);
  long long acc[L_N + C_N];
#pragma unroll
  for (int i = 0; i < L_N + C_N; ++i) acc[i] = 0;
  for (long long t = (long long)bm.lb * kBlock + threadIdx.x; t < tot; t += (long long)bm.nb * kBlock) {
    const long long slot = n0 + t;
    if (slot >= R.capacity) {   // never write past the particle arrays; counted
      acc[L_N + C_INJ_LOST] += 1;
      continue;
    }
    int s = 0;
    long long off = 0;
    while (s < R.nsrc - 1 && t >= off + cnt[s]) { off += cnt[s]; ++s; }
    const gptr<const SourceDesc> S = G(R.src) + s;
    const uint32_t id = (uint32_t)(first[s] + (t - off));
    const Uni4<T> a = draws<T>(id, R.seed, step, SLOT_INJ_A);
    const Uni4<T> b = draws<T>(id, R.seed, step, SLOT_INJ_B);
    int cy, cz;
    T oy, oz, eps, omc, wn;
    if (S->kind == 1) {
      // the paper's envelope: a face cell from the list, position uniform
      // over it, mean energy a0 sqrt(f g), Moore-scaling cone, eq. N_cell weight
      const int cell = G(S->cells)[(int)((t - off) / S->per_cell)];
      const int j = cell & 0xFFFF, k = cell >> 16;
      const T qr = (T)2 * m_sqrt(((T)j + (T)0.5 - (T)S->y0) * ((T)j + (T)0.5 - (T)S->y0) +
                                 ((T)k + (T)0.5 - (T)S->z0) * ((T)k + (T)0.5 - (T)S->z0)) / (T)S->rf;
      const T qt = (T)2 * ((T)step + (T)0.5 - (T)S->tp) / (T)S->tf;
      const T ln2 = (T)0.69314718055994530942;
      const T sq = m_sqrt(m_exp(-qr * qr * ln2) * m_exp(-qt * qt * ln2));
      cy = j; oy = a.a;
      cz = k; oz = a.b;
      eps = -(T)S->a0 * sq * m_log((T)1 - a.c);
      const T th_moore = m_atan(m_sqrt((T)2 / eps));
      omc = (T)1 - m_cos(th_moore < (T)S->cap ? th_moore : (T)S->cap);
      wn = (T)S->wn * sq;
    } else if (S->kind == 2) {
      // mono-energetic beam along +x, every face cell, uniform over the cell
      const long long cidx = (t - off) / S->per_cell;
      cy = (int)(cidx % R.ny); oy = a.a;
      cz = (int)(cidx / R.ny); oz = a.b;
      eps = (T)S->t_hot;
      omc = (T)0;
      wn = (T)S->wn;
    } else {
      const T r = m_sqrt((T)-2 * (T)S->sig2 * m_log((T)1 - (T)0.5 * a.a));
      T sps, cps;
      m_sincos2pi(a.b, sps, cps);
      to_cell((T)S->y0 + r * cps, R.ny, cy, oy);
      to_cell((T)S->z0 + r * sps, R.nz, cz, oz);
      eps = -(T)S->t_hot * m_log((T)1 - a.c);
      omc = (T)S->one_minus_cos;
      wn = (T)S->wn;
    }
    const T ct = (T)1 - a.d * omc;
    T st2 = (T)1 - ct * ct;
    const T st = m_sqrt(st2 > (T)0 ? st2 : (T)0);
    T spc, cpc;
    m_sincos2pi(b.a, spc, cpc);
    const T um = umag_of(eps);
    const T ux = um * ct, uy = um * st * cpc, uz = um * st * spc;
    const T tau = -m_log((T)1 - b.b);
    P.cell[slot] = pack_cell(R.ix_lo, cy, cz);
    P.ox[slot] = (T)0;
    P.oy[slot] = oy;
    P.oz[slot] = oz;
    P.ux[slot] = ux;
    P.uy[slot] = uy;
    P.uz[slot] = uz;
    P.wn[slot] = wn;
    P.tau[slot] = tau;
    P.id[slot] = id;
    if (R.physics & PHYS_DELTA) P.taud[slot] = -m_log((T)1 - b.c);
    const T u2 = ux * ux + uy * uy + uz * uz;
    acc[L_INJECTED] += to_fixed(kinetic(u2, m_sqrt((T)1 + u2)) * wn * (T)kLedScale);
    acc[L_N + C_INJECTED] += 1;
  }
  block_flush<L_N, C_N>(acc, R.acc_led, R.events);
}

// ---------------------------------------------------------------------------
// Yee stencil helpers.  Along an axis a node quantity uses indices (c, c+1)
// with weights (1-o, o); a staggered quantity sits at half-integers and uses
// (c-1, c) or (c, c+1).  A staggered index one past either end is the mirror
// ghost of the nearest index, with the opposite sign: its weight joins that
// index's, and the pair keeps i1 = i0 + 1 with a zero weight on the other
// (an index inside the node-sized arrays), so that the two values of a pair
// are always neighbours in memory and load together.
// ---------------------------------------------------------------------------
template <typename T>
struct Axis { int i0, i1; T w0, w1; };

template <typename T>
__device__ __forceinline__ Axis<T> node_axis(int c, T o) { return Axis<T>{c, c + 1, (T)1 - o, o}; }

template <typename T>
__device__ __forceinline__ Axis<T> stag_axis(int c, T o, int n) {
  Axis<T> a;
  T f;
  if (o >= (T)0.5) { a.i0 = c; f = o - (T)0.5; }
  else { a.i0 = c - 1; f = o + (T)0.5; }
  a.w0 = (T)1 - f;
  a.w1 = f;
  if (a.i0 < 0) { a.i0 = 0; a.w0 = a.w1 - a.w0; a.w1 = (T)0; }     // ghost at -1: odd image of 0
  else if (a.i0 + 1 > n - 1) { a.w0 = a.w0 - a.w1; a.w1 = (T)0; }  // ghost at n: odd image of n - 1
  a.i1 = a.i0 + 1;
  return a;
}

template <typename T>
__device__ __forceinline__ T gather8(gptr<const T> F, int sx, int sxy, const Axis<T>& ax,
                                     const Axis<T>& ay, const Axis<T>& az) {
  const int r00 = ay.i0 * sx + az.i0 * sxy, r10 = ay.i1 * sx + az.i0 * sxy;
  const int r01 = ay.i0 * sx + az.i1 * sxy, r11 = ay.i1 * sx + az.i1 * sxy;
  const T v00 = ax.w0 * F[r00 + ax.i0] + ax.w1 * F[r00 + ax.i1];
  const T v10 = ax.w0 * F[r10 + ax.i0] + ax.w1 * F[r10 + ax.i1];
  const T v01 = ax.w0 * F[r01 + ax.i0] + ax.w1 * F[r01 + ax.i1];
  const T v11 = ax.w0 * F[r11 + ax.i0] + ax.w1 * F[r11 + ax.i1];
  return az.w0 * (ay.w0 * v00 + ay.w1 * v10) + az.w1 * (ay.w0 * v01 + ay.w1 * v11);
}

// The same from a 6^3-node halo in LDS whose first node is (bx, by, bz).
template <typename T>
__device__ __forceinline__ T gather8_lds(const T* __restrict__ F, int bx, int by, int bz, const Axis<T>& ax,
                                         const Axis<T>& ay, const Axis<T>& az) {
  const int i0 = ax.i0 - bx, i1 = ax.i1 - bx;
  const int j0 = (ay.i0 - by) * kHalo, j1 = (ay.i1 - by) * kHalo;
  const int k0 = (az.i0 - bz) * kHalo * kHalo, k1 = (az.i1 - bz) * kHalo * kHalo;
  const T v00 = ax.w0 * F[j0 + k0 + i0] + ax.w1 * F[j0 + k0 + i1];
  const T v10 = ax.w0 * F[j1 + k0 + i0] + ax.w1 * F[j1 + k0 + i1];
  const T v01 = ax.w0 * F[j0 + k1 + i0] + ax.w1 * F[j0 + k1 + i1];
  const T v11 = ax.w0 * F[j1 + k1 + i0] + ax.w1 * F[j1 + k1 + i1];
  return az.w0 * (ay.w0 * v00 + ay.w1 * v10) + az.w1 * (ay.w0 * v01 + ay.w1 * v11);
}

// ---------------------------------------------------------------------------
// reflux / escape on one axis (Sec. II.A).  Returns false if the electron
// leaves the simulation.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ bool boundary_axis(const RunDesc& R, int axis, int& c, T& o, int lo, int hi,
                                              T& ux, T& uy, T& uz, T& eps, T wn, uint32_t id,
                                              long long step, long long* led) {
  const bool below = c < lo;
  const bool above = c >= hi;
  if (!(below || above)) return true;
  const int mode = R.bc[axis];   // 0 reflux, 1 open, 2 mirror, 3 periodic
  if (mode == 3) {   // re-enter through the opposite wall; nothing else changes
    const int n = hi - lo;
    c = lo + ((c - lo) % n + n) % n;
    return true;
  }
  if (mode == 1 || (mode == 0 && eps > (T)R.eps_esc)) {
    lds_add(&led[L_ESCAPED], to_fixed(eps * wn * (T)kLedScale));
    lds_add(&led[L_N + C_ESCAPED], 1LL);
    return false;
  }
  // mirror about the face, then clamp into [lo, hi)
  int c2 = (below ? 2 * lo : 2 * hi) - c - 1;
  T o2 = (T)1 - o;
  if (o2 >= (T)1) { c2 += 1; o2 = (T)0; }
  if (c2 < lo) { c2 = lo; o2 = (T)0; }
  if (c2 >= hi) { c2 = hi - 1; o2 = (T)1 - (T)(sizeof(T) == 4 ? 5.9604644775390625e-08 : 1.1102230246251565e-16); }
  c = c2;
  o = o2;
  if (axis == 0) ux = -ux;
  else if (axis == 1) uy = -uy;
  else uz = -uz;
  if (mode == 2) return true;   // specular wall: nothing else changes
  lds_add(&led[L_N + C_REFLUX], 1LL);
  // energy or momentum loss
  const T um = m_sqrt(ux * ux + uy * uy + uz * uz);
  T scale;
  if (R.reflux_ke_mode) {
    // an electron already stopped by the collisions (u = 0) stays at rest
    scale = um > (T)0 ? umag_of(eps * (T)R.keep_frac) / um : (T)0;
  } else {
    const T um2 = um - (T)R.du_tnsa;
    if (!(um2 > (T)0)) {
      lds_add(&led[L_REFLUX], to_fixed(eps * wn * (T)kLedScale));
      return false;
    }
    scale = um2 / um;
  }
  ux *= scale; uy *= scale; uz *= scale;
  const T u2 = ux * ux + uy * uy + uz * uz;
  const T eps_a = kinetic(u2, m_sqrt((T)1 + u2));
  lds_add(&led[L_REFLUX], to_fixed((eps - eps_a) * wn * (T)kLedScale));
  eps = eps_a;
  if (u2 > (T)0) {
    const Uni4<T> rd = draws<T>(id, R.seed, step, SLOT_REFLUX0 + (uint32_t)axis);
    rotate(ux, uy, uz, (rd.a - (T)0.5) * (T)R.sigma_dth, rd.b);
    const T v2 = ux * ux + uy * uy + uz * uz;
    const T eps_r = kinetic(v2, m_sqrt((T)1 + v2));
    lds_add(&led[L_RESIDUAL], to_fixed((eps - eps_r) * wn * (T)kLedScale));
    eps = eps_r;
  }
  // leave the face inwards
  if (axis == 0) ux = below ? fabs(ux) : -fabs(ux);
  else if (axis == 1) uy = below ? fabs(uy) : -fabs(uy);
  else uz = below ? fabs(uz) : -fabs(uz);
  return true;
}

// ---------------------------------------------------------------------------
// LDS staging of one chunk of particles.  Particles sorted by tile arrive in
// chunks of kBlock; the chunk's most populated tiles (up to kRegions) are its
// regions.  Deposits of an electron in a region tile go to LDS integer
// accumulators covering the 6x6x6 nodes that tile's stencils can reach and
// its 4x4x4 cells of collisional heat; the two most populated regions also
// stage their field halos for the gather; destinations are counted in the
// 5x5x5 tiles around the most populated one, where its electrons can move in
// one step; everything else falls back to global gathers and atomics.  A
// region's sums go to HBM as its tile's partials (plain stores) if this
// workgroup holds the tile's claim for the step, else with one atomic per
// non-zero entry into the accumulators; k_gather adds both into j_h.
// ---------------------------------------------------------------------------
// Current contributions are fixed point.  FP64 runs use 2^40 units per
// (e w_ref c / dx^3) in 64-bit LDS words.  FP32-mixed runs round each
// contribution to 2^20 units and sum them in 32-bit LDS words (and partials),
// widened to the 2^40 HBM accumulators at the flush or in the gather.  Every contribution is rounded the same
// way whether it goes through LDS or straight to HBM, so the sums stay
// independent of the electron order.
//
// A region whose tile recurs in the workgroup's next chunk carries its sums
// over (dense tiles span many chunks), for at most JAcc::max_chunks chunks
// before a flush.  Bounds: a chunk adds at most kBlock contributions to a
// word; FP32: each of magnitude at most 2^21 (w / w_ref <= 2), 3 chunks stay
// below 2^31; FP64: each below 2^46 (w / w_ref <= 64), 31 chunks below 2^59.
template <typename T> struct JAcc {
  using type = long long;
  static constexpr int shift = 0, max_chunks = 31;
};
template <> struct JAcc<float> {
  using type = int;
  static constexpr int shift = 20, max_chunks = 3;
};
static_assert((long long)JAcc<float>::max_chunks * kBlock * 2 * (1LL << (40 - JAcc<float>::shift)) < (1LL << 31),
              "FP32 LDS current sums could wrap");
static_assert((long long)JAcc<double>::max_chunks * kBlock * 64 * (1LL << 40) < (1LL << 62),
              "FP64 LDS current sums could wrap");
constexpr int kRegions = 6;    // LDS regions per chunk
constexpr int kKeys = 64;      // census keys of a chunk's tiles (one per lane of a wave)
constexpr int kLdsTab = 128;   // table rows staged in LDS

// A tile's 216 halo nodes split into 27 parts by the tile that owns the
// node: part e (a step of -1, 0 or +1 per axis, index (ex + 1) + 3 (ey + 1)
// + 9 (ez + 1); 13 is the tile itself) holds the halo layer 0 (e = -1) or 5
// (e = +1) on its fixed axes and layers 1..4 on the others, x fastest.  The
// deposit of current component c reaches layer 0 only along axis c (its
// stencil is staggered there, node-centred on the other axes), so c's
// partials hold the 150 nodes of the parts without e = -1 on another axis.
// A tile's partials (pj: [tile][component][150]) list those parts one after
// the other, part 13 first: position p of component c is halo node l[c][p]
// (x + 6 y + 36 z), part e starts at off[c][e] (-1: none).  The gather of a
// tile reads the part of each neighbour that lies in it as one run of words.
struct PjPerm {
  unsigned char l[3][kPjWords];
  short off[3][27];
};
__host__ __device__ constexpr int pj_layer(int e, int o) { return e < 0 ? 0 : (e > 0 ? kHalo - 1 : 1 + o); }
constexpr PjPerm make_pj_perm() {
  PjPerm P{};
  for (int c = 0; c < 3; ++c) {
    int pos = 0;
    for (int pass = 0; pass < 2; ++pass)
      for (int e = 0; e < 27; ++e) {
        if ((pass == 0) != (e == 13)) continue;
        const int ed[3] = {e % 3 - 1, (e / 3) % 3 - 1, e / 9 - 1};
        P.off[c][e] = -1;
        if ((c != 0 && ed[0] < 0) || (c != 1 && ed[1] < 0) || (c != 2 && ed[2] < 0)) continue;
        P.off[c][e] = (short)pos;
        for (int oz = 0; oz < (ed[2] ? 1 : kTile); ++oz)
          for (int oy = 0; oy < (ed[1] ? 1 : kTile); ++oy)
            for (int ox = 0; ox < (ed[0] ? 1 : kTile); ++ox)
              P.l[c][pos++] =
                  (unsigned char)(pj_layer(ed[0], ox) + kHalo * (pj_layer(ed[1], oy) + kHalo * pj_layer(ed[2], oz)));
      }
  }
  return P;
}
__constant__ PjPerm kPjPerm = make_pj_perm();
static_assert(make_pj_perm().off[0][13] == 0 && make_pj_perm().l[2][kPjWords - 1] == kHaloN - 1 &&
                  make_pj_perm().off[1][0] < 0 && make_pj_perm().off[0][12] >= 0 && make_pj_perm().off[1][12] < 0,
              "halo order");

// Word, inside the partials of tile u = v - e, of component c of own node o
// of tile v, which u holds in its part e (indexed by o over the axes where
// e is 0); -1 where component c has no such part.
__device__ __forceinline__ int pj_word(int ex, int ey, int ez, int c, int ox, int oy, int oz) {
  int idx = 0, sc = 1;
  if (!ex) { idx += ox; sc = kTile; }
  if (!ey) { idx += oy * sc; sc *= kTile; }
  if (!ez) idx += oz * sc;
  const int off = kPjPerm.off[c][(ex + 1) + 3 * (ey + 1) + 9 * (ez + 1)];
  return off < 0 ? -1 : c * kPjWords + off + idx;
}

// The per-tile counts that pick the regions use slots that alternate between
// chunks, so that counting the next chunk never races the reads of this one.
template <typename T>
struct ChunkLds {
  typename JAcc<T>::type J[kRegions][3 * kHaloN];
  long long heat[kRegions][kTile * kTile * kTile];
  unsigned cnt[kNbN];
  int tc[2][kKeys], tt[2][kKeys];   // electrons per tile of a chunk, by census key, and the tile
  long long led[L_N + C_N];   // rare ledger terms and event counts of the block
  T ph[6][kBlock];            // emitted photon of each lane: k, u (3), |u|, gamma
  T tsig[kLdsTab], tsub[kLdsTab];   // cross-section columns of the tables, if they fit
  T F[2][6][kHaloN];                // E, B on the 6^3-node halos of the two fullest regions
  int own[kRegions];                // the region's tile was first claimed this step by this workgroup
  unsigned char perm[3 * kPjWords]; // halo node of each position of the partials (kPjPerm.l)
};

struct Home {
  int ok;                 // the tile exists (the chunk has an alive electron)
  int tx, ty, tz;         // home tile
  int bx, by, bz;         // first node of the home tile's halo
};

__device__ __forceinline__ int tile_of(const RunDesc& R, int i, int j, int k) {
  return (i >> 2) + R.ntx * ((j >> 2) + R.nty * (k >> 2));
}

__device__ __forceinline__ Home make_home(const RunDesc& R, int t) {
  Home h;
  h.ok = t >= 0 && t != kNoTile;
  if (!h.ok) t = 0;
  const uint32_t q = R.fd_tx.div((uint32_t)t), z = R.fd_ty.div(q);
  h.tx = t - (int)q * R.ntx;
  h.ty = (int)q - (int)z * R.nty;
  h.tz = (int)z;
  h.bx = kTile * h.tx - 1;
  h.by = kTile * h.ty - 1;
  h.bz = kTile * h.tz - 1;
  return h;
}

// bin of tile (tx,ty,tz) in the 5x5x5 neighbourhood of home, or -1
__device__ __forceinline__ int nb_bin(const Home& h, int tx, int ty, int tz) {
  const int dx = tx - h.tx + 2, dy = ty - h.ty + 2, dz = tz - h.tz + 2;
  if ((unsigned)dx >= (unsigned)kNb || (unsigned)dy >= (unsigned)kNb || (unsigned)dz >= (unsigned)kNb) return -1;
  return dx + kNb * (dy + kNb * dz);
}

template <typename T>
__device__ __forceinline__ void lds_init(ChunkLds<T>& L) {
  for (int t = threadIdx.x; t < kRegions * 3 * kHaloN; t += kBlock) (&L.J[0][0])[t] = 0;
  for (int t = threadIdx.x; t < kRegions * kTile * kTile * kTile; t += kBlock) (&L.heat[0][0])[t] = 0;
  if (threadIdx.x < kNbN) L.cnt[threadIdx.x] = 0;
  if (threadIdx.x < 2 * kKeys) { (&L.tc[0][0])[threadIdx.x] = 0; (&L.tt[0][0])[threadIdx.x] = -1; }
  if (threadIdx.x < L_N + C_N) L.led[threadIdx.x] = 0;
  for (int t = threadIdx.x; t < 3 * kPjWords; t += kBlock) L.perm[t] = (&kPjPerm.l[0][0])[t];
}

// Moves the LDS sums of one region to HBM and clears them for the next
// chunk: the tile's partials as whole lines of plain stores if this
// workgroup holds the tile's claim of the step, else one atomic per
// non-zero entry into the accumulators (the tile marked for the gather).
template <typename T>
__device__ __forceinline__ void lds_flush_region(const RunDesc& R, ChunkLds<T>& L, int r, int tile, int stampv) {
  using A = typename JAcc<T>::type;
  A* J = L.J[r];
  if (L.own[r]) {
    A* const dst = (A*)R.pj + (long long)tile * (3 * kPjWords);
    for (int t = threadIdx.x; t < 3 * kPjWords; t += kBlock) {
      const int c = t >= 2 * kPjWords ? 2 : (t >= kPjWords ? 1 : 0);
      A* w = &J[c * kHaloN + L.perm[t]];
      dst[t] = *w;
      *w = 0;
    }
    if (threadIdx.x < kTile * kTile * kTile) {
      R.ph[(long long)tile * (kTile * kTile * kTile) + threadIdx.x] = L.heat[r][threadIdx.x];
      L.heat[r][threadIdx.x] = 0;
    }
    return;
  }
  const Home h = make_home(R, tile);
  const int sx = R.nx + 1, sxy = (R.nx + 1) * (R.ny + 1);
  if (threadIdx.x == 0) G(R.tdirty)[tile] = stampv;
  for (int t = threadIdx.x; t < 3 * kHaloN; t += kBlock) {
    long long v = (long long)J[t];
    if (v == 0) continue;
    J[t] = 0;
    v *= (1LL << JAcc<T>::shift);
    const int c = t / kHaloN, l = t % kHaloN;
    const int i = h.bx + l % kHalo, j = h.by + (l / kHalo) % kHalo, k = h.bz + l / (kHalo * kHalo);
    if (i < 0 || j < 0 || k < 0 || i > R.nx || j > R.ny || k > R.nz) continue;
    atomic_add_i64(&R.Jacc[c][i + sx * j + sxy * k], v);
  }
  if (threadIdx.x < kTile * kTile * kTile) {
    const long long v = L.heat[r][threadIdx.x];
    const int l = threadIdx.x;
    const int i = kTile * h.tx + (l & 3), j = kTile * h.ty + ((l >> 2) & 3), k = kTile * h.tz + (l >> 4);
    if (v != 0) {
      L.heat[r][threadIdx.x] = 0;
      if (i < R.nx && j < R.ny && k < R.nz) atomic_add_i64(&R.heat_acc[i + R.nx * (j + R.ny * k)], v);
    }
  }
}

// Destination counts of chunk ch (bins around home tile h) to the tile
// counters, cleared.  The counter's old value is the chunk's offset inside
// the tile; it is stored one chunk later (pend_*), when the atomic is back.
template <typename T>
__device__ __forceinline__ void lds_flush_counts(const RunDesc& R, ChunkLds<T>& L, const Home& h, long long ch,
                                                 unsigned& pend_val, long long& pend_at) {
  if (threadIdx.x < kNbN) {
    const unsigned v = L.cnt[threadIdx.x];
    L.cnt[threadIdx.x] = 0;
    const int l = threadIdx.x;
    const int tx = h.tx + l % kNb - 2, ty = h.ty + (l / kNb) % kNb - 2, tz = h.tz + l / (kNb * kNb) - 2;
    if (v != 0 && tx >= 0 && ty >= 0 && tz >= 0 && tx < R.ntx && ty < R.nty && tz < R.ntz) {
      pend_val = atomic_add_u32(&R.tile_cnt[tx + R.ntx * (ty + R.nty * tz)], v);
      pend_at = ch * kNbN + l;
    }
  }
}

// deposit of one current component: 8 corners to LDS (a home tile) or HBM
__device__ __forceinline__ long long jfix(double x) { return to_fixed(x); }
__device__ __forceinline__ int jfix(float x) { return __float2int_rn(x); }

// Js: the component's LDS block of the electron's home region (first halo
// node bx, by, bz), or null for a deposit straight to HBM.
template <typename T>
__device__ __forceinline__ void deposit8(long long* __restrict__ J, typename JAcc<T>::type* __restrict__ Js,
                                         int bx, int by, int bz, int sx, int sxy, const Axis<T>& ax,
                                         const Axis<T>& ay, const Axis<T>& az, T amp) {
  using A = typename JAcc<T>::type;
  const T a00 = amp * az.w0 * ay.w0, a10 = amp * az.w0 * ay.w1;
  const T a01 = amp * az.w1 * ay.w0, a11 = amp * az.w1 * ay.w1;
  const A v[8] = {jfix(a00 * ax.w0), jfix(a00 * ax.w1), jfix(a10 * ax.w0), jfix(a10 * ax.w1),
                  jfix(a01 * ax.w0), jfix(a01 * ax.w1), jfix(a11 * ax.w0), jfix(a11 * ax.w1)};
  if (Js) {
    const int i0 = ax.i0 - bx, i1 = ax.i1 - bx;
    const int j0 = (ay.i0 - by) * kHalo, j1 = (ay.i1 - by) * kHalo;
    const int k0 = (az.i0 - bz) * kHalo * kHalo, k1 = (az.i1 - bz) * kHalo * kHalo;
    lds_add(&Js[i0 + j0 + k0], v[0]);
    lds_add(&Js[i1 + j0 + k0], v[1]);
    lds_add(&Js[i0 + j1 + k0], v[2]);
    lds_add(&Js[i1 + j1 + k0], v[3]);
    lds_add(&Js[i0 + j0 + k1], v[4]);
    lds_add(&Js[i1 + j0 + k1], v[5]);
    lds_add(&Js[i0 + j1 + k1], v[6]);
    lds_add(&Js[i1 + j1 + k1], v[7]);
  } else {
    constexpr long long up = 1LL << JAcc<T>::shift;
    const int r00 = ay.i0 * sx + az.i0 * sxy, r10 = ay.i1 * sx + az.i0 * sxy;
    const int r01 = ay.i0 * sx + az.i1 * sxy, r11 = ay.i1 * sx + az.i1 * sxy;
    atomic_add_i64(&J[r00 + ax.i0], (long long)v[0] * up);
    atomic_add_i64(&J[r00 + ax.i1], (long long)v[1] * up);
    atomic_add_i64(&J[r10 + ax.i0], (long long)v[2] * up);
    atomic_add_i64(&J[r10 + ax.i1], (long long)v[3] * up);
    atomic_add_i64(&J[r01 + ax.i0], (long long)v[4] * up);
    atomic_add_i64(&J[r01 + ax.i1], (long long)v[5] * up);
    atomic_add_i64(&J[r11 + ax.i0], (long long)v[6] * up);
    atomic_add_i64(&J[r11 + ax.i1], (long long)v[7] * up);
  }
}

// Ranks of the lanes in their bins (b < 0: none), taken in lane order from
// the block's LDS counters: one LDS atomic per distinct bin of the wave, so
// lanes of one bin get consecutive ranks and their writes coalesce.  Every
// lane of the wave takes part; the leader's values are read with readlane.
__device__ __forceinline__ unsigned wave_rank(unsigned* cnt, int b) {
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1ull;
  unsigned rank = 0;
  unsigned long long todo = __ballot(b >= 0);
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int lb = __builtin_amdgcn_readlane(b, leader);
    const unsigned long long m = __ballot(b == lb);
    unsigned base = 0;
    if (lane == leader) base = atomicAdd(&cnt[lb], (unsigned)__popcll(m));
    base = (unsigned)__builtin_amdgcn_readlane((int)base, leader);
    if (b == lb) rank = base + (unsigned)__popcll(m & below);
    todo &= ~m;
  }
  return rank;
}

// Tally of one photon (Sec. II.C, Table I bins): emitted at energy k about
// the electron direction u (|u| = um, Lorentz factor g), weight wn / boost.
// Returns the emitting electron's new optical depth, drawn from the same
// variates.
template <typename T>
__device__ __forceinline__ T photon_tally(const RunDesc& R, ChunkLds<T>& S, T wn, uint32_t id, long long step) {
  const int t = threadIdx.x;
  const T kph = S.ph[0][t], um = S.ph[4][t], g = S.ph[5][t];
  T dxp = S.ph[1][t], dyp = S.ph[2][t], dzp = S.ph[3][t];
  const Uni4<T> pd = draws<T>(id, R.seed, step, SLOT_PHOTON);
  // photon direction about the electron direction: theta = u / gamma, u from
  // the Tsai-based mixture of Gamma(2) laws of rates a = 0.625 (weight 1/4)
  // and 3a (weight 3/4), -ln(r1 r2) / rate; draw a picks the law and, rescaled
  // onto (0, 1), serves as r1
  const bool first = pd.a < (T)0.25;
  const T r1 = first ? pd.a / (T)0.25 : (pd.a - (T)0.25) / (T)0.75;
  T th = -m_log(r1 * pd.d) / ((first ? (T)0.625 : (T)1.875) * g);
  th = th < (T)kPi ? th : (T)kPi;
  rotate(dxp, dyp, dzp, th, pd.b);
  T cx = dxp / um;
  cx = cx > (T)1 ? (T)1 : (cx < (T)-1 ? (T)-1 : cx);
  const T tq = m_acos(cx) * (T)R.nth * (T)(1.0 / kPi);
  const int it = tq >= (T)0 ? (tq < (T)(R.nth - 1) ? (int)tq : R.nth - 1) : 0;
  const T eq = (m_log(kph) - (T)R.ln_Elo) * (T)R.e_bin_scale;
  const int ie = !(eq >= (T)0) ? -1 : (eq >= (T)R.nE ? R.nE : (int)eq);
  const T wph = wn * (T)R.inv_boost;
  const long long vE = to_fixed(kph * wph * (T)kLedScale);
  const long long vN = to_fixed(wph * (T)kLedScale);
  const int nbin = R.nE * R.nth;
  long long* hist = R.acc_hist + (blockIdx.x & (kHistCopies - 1)) * R.hist_stride;
  if (ie < 0) {
    atomic_add_i64(&hist[2 * nbin + 0], vE);
    atomic_add_i64(&hist[2 * nbin + 1], vN);
  } else if (ie >= R.nE) {
    atomic_add_i64(&hist[2 * nbin + 2], vE);
    atomic_add_i64(&hist[2 * nbin + 3], vN);
  } else {
    atomic_add_i64(&hist[ie * R.nth + it], vE);
    atomic_add_i64(&hist[nbin + ie * R.nth + it], vN);
  }
  if (kph >= (T)R.Ethr) lds_add(&S.led[L_PHOTON_THR], vE);
  lds_add(&S.led[L_RAD_D], vE);
  lds_add(&S.led[L_N + C_EMITTED], 1LL);
  return -m_log((T)1 - pd.c);   // the electron's next optical depth
}

// XCD-aware chunk range of a workgroup: workgroup b runs on XCD b % 8, so
// each XCD gets one contiguous eighth of the (tile-sorted) chunks.
struct ChunkRange { long long beg, end, stride; };

// The same eighth cut into one contiguous run of chunks per workgroup (a
// tile split between two chunks then stays in one workgroup's LDS).
__device__ __forceinline__ ChunkRange chunk_run(const BlockMap& bm, long long n) {
  const long long nch = (n + kBlock - 1) / kBlock;
  const long long per = (nch + 7) >> 3;
  const int xcd = bm.lb & 7;
  const long long lo = (long long)xcd * per, hi = lo + per < nch ? lo + per : nch;
  const long long nbx = bm.nb >> 3, q = bm.lb >> 3;
  const long long m = (hi - lo + nbx - 1) / nbx;
  ChunkRange r;
  r.beg = lo + q * m;
  r.end = r.beg + m < hi ? r.beg + m : hi;
  r.stride = 1;
  return r;
}

__device__ __forceinline__ ChunkRange chunk_range(const BlockMap& bm, long long n) {
  const long long nch = (n + kBlock - 1) / kBlock;
  const long long per = (nch + 7) >> 3;
  const int xcd = bm.lb & 7;
  ChunkRange r;
  r.beg = (long long)xcd * per + (bm.lb >> 3);
  r.end = (long long)xcd * per + per < nch ? (long long)xcd * per + per : nch;
  r.stride = bm.nb >> 3;
  return r;
}

// ---------------------------------------------------------------------------
// delta rays (App. B): restricted loss below the cut, Moller scatter above
// ---------------------------------------------------------------------------
// Restricted continuous loss over the step [m c^2] of an electron of
// kinetic energy t, Lorentz factor g, u^2 = (beta gamma)^2: c_rst L / beta,
// L = ln(2 (g + 1)) - 2 ln(I) + F^-(t, D) - delta, D = min(cut, t / 2),
// F^- = -1 - beta^2 + ln((t - D) D) + t / (t - D) + (D^2/2 + (2t + 1) ln(1 - D/t)) / g^2,
// delta = max(0, d_dens0 + ln u^2); L clamped at zero.
template <typename T>
__device__ __forceinline__ T restricted_loss(const RunDesc& R, T t, T g, T u2) {
  const T ig = (T)1 / g;
  const T b2 = u2 * ig * ig;
  const T hc = (T)0.5 * t;
  const T D = (T)R.d_cut < hc ? (T)R.d_cut : hc;
  // ln(2 (g + 1)) + ln((t - D) D) as one logarithm
  T L = m_log((T)2 * (g + (T)1) * (t - D) * D) - (T)R.d_lnI2 - (T)1 - b2 + t / (t - D) +
        ((T)0.5 * D * D + ((T)2 * t + (T)1) * m_log1p(-D / t)) * ig * ig;
  // the density effect is zero below (beta gamma)^2 = exp(-d_dens0)
  if (u2 > (T)R.d_u2min) L -= (T)R.d_dens0 + m_log(u2);
  L = L > (T)0 ? L : (T)0;
  return (T)R.c_rst * L / m_sqrt(b2);
}

// x^2 times the bracket of the Moller cross-section d sigma / dx, with
// a = (2g - 1)/g^2, b = ((g - 1)/g)^2; convex on (0, 1/2]
template <typename T>
__device__ __forceinline__ T moller_g(T x, T a, T b) {
  const T y = (T)1 - x;
  const T xx = x * x;
  return b * xx + (T)1 - a * x + xx / (y * y) - a * xx / y;
}

// ---------------------------------------------------------------------------
// Urban-type elastic scatter (App. B): model functions of the polar angle
// whose first two Legendre moments are Lewis theory's
// ---------------------------------------------------------------------------
// L(a) = coth a - 1/a, C = 1 - L, S = L - a/3 and dL/da, in double: below
// 1/2 the Taylor series sum 2^2n B_2n a^(2n-1) / (2n)! (twelve terms), above
// C = 1/a - 2 / (e^2a - 1) (no cancellation as C -> 0).
__device__ __forceinline__ void langevin_d(double a, double& L, double& C, double& S, double& dL) {
  if (a < 0.5) {
    const double q = a * a;
    // coefficients of a^3, a^5, ..., a^23
    const double c2 = -1.0 / 45.0, c3 = 2.0 / 945.0, c4 = -1.0 / 4725.0, c5 = 2.0 / 93555.0,
                 c6 = -1382.0 / 638512875.0, c7 = 4.0 / 18243225.0, c8 = -3617.0 / 162820783125.0,
                 c9 = 87734.0 / 38979295480125.0, c10 = -349222.0 / 1531329465290625.0,
                 c11 = 310732.0 / 13447856940643125.0, c12 = -472728182.0 / 201919571963756521875.0;
    const double p = c2 + q * (c3 + q * (c4 + q * (c5 + q * (c6 + q * (c7 + q * (c8 + q * (c9 +
                     q * (c10 + q * (c11 + q * c12)))))))));
    S = a * q * p;
    L = a * (1.0 / 3.0) + S;
    C = 1.0 - L;
    dL = 1.0 / 3.0 + q * (3 * c2 + q * (5 * c3 + q * (7 * c4 + q * (9 * c5 + q * (11 * c6 +
         q * (13 * c7 + q * (15 * c8 + q * (17 * c9 + q * (19 * c10 + q * (21 * c11 + q * 23 * c12))))))))));
  } else {
    const double e = expm1(2.0 * a);   // inf above a ~ 354: 2 / e -> 0
    C = 1.0 / a - 2.0 / e;
    L = 1.0 - C;
    S = L - a * (1.0 / 3.0);
    // 1 / sinh^2 a = 4 (e + 1) / e^2, negligible against 1/a^2 far out
    dL = a < 40.0 ? 1.0 / (a * a) - 4.0 * (e + 1.0) / (e * e) : 1.0 / (a * a);
  }
}

// Root in t = ln a of a residual that decreases in a, from t: Newton steps
// kept inside the bracket, bisection where a step leaves it.  f(t, F, dF/dt).
// Newton converges quadratically, so a step below 1e-9 leaves an error of
// order 1e-18 and ends the search.
template <class Fn>
__device__ __forceinline__ double urban_solve(Fn f, double t) {
  double lo = -41.0, hi = 41.0;
  t = t > lo ? (t < hi ? t : hi) : lo;
#pragma unroll 1
  for (int it = 0; it < 100; ++it) {
    double F, dF;
    f(t, F, dF);
    if (F == 0.0) break;
    if (F > 0.0) lo = t; else hi = t;
    double tn = t - F / dF;
    const bool newton = tn > lo && tn < hi;
    if (!newton) tn = 0.5 * (lo + hi);
    const double step = fabs(tn - t);
    t = tn;
    if ((newton && step < 1e-9 * (fabs(t) > 1.0 ? fabs(t) : 1.0)) || hi - lo < 1e-15) break;
  }
  return t;
}

// 1 - cos theta of one step's deflection of an electron of u^2 = (p/(m c))^2:
// x_l = v dt / lambda_l summed over the elements from the screened Rutherford
// law, sigma_1 = 8 pi k (ln(1 + 1/A) - 1/(1 + A)), sigma_2 = 24 pi k ((1 + 2A)
// ln(1 + 1/A) - 2); the model function (1 - w_i) a e^(-a (1 - cos)) / (1 -
// e^(-2a)) + w_i / 2 with 1/L(a) - 3/a = exp(x_1 - x_2) and w_i = 1 -
// exp(-x_1) / L(a), or, where that w_i < 0, w_i = 0 and L(a) = exp(-x_1).
// Quantities near 1 are carried as their distance from 1.
// ua < w_i picks the isotropic part; ub gives the angle by the part's inverse CDF.
__device__ __forceinline__ double urban_one_minus_cos(const RunDesc& R, double u2, double ua, double ub) {
  const double b2 = u2 / (1.0 + u2);
  double x1 = 0.0, x2 = 0.0;
#pragma unroll 1
  for (int j = 0; j < R.u_n; ++j) {
    const double A = R.u_ca[j] * (1.0 + R.u_cb[j] / b2) / u2;
    const double lg = log1p(1.0 / A);
    x1 += R.u_k1[j] * (lg - 1.0 / (1.0 + A));
    x2 += R.u_k1[j] * ((1.0 + 2.0 * A) * lg - 2.0);
  }
  const double iv = 1.0 / (u2 * sqrt(b2));
  x1 *= iv;
  x2 *= 3.0 * iv;
  const double d = x2 - x1;
  const double r = exp(-d), rho = -expm1(-d);
  // psi(a) = 1 - (1/L - 3/a) against rho = 1 - r: large a as 3/a - c/(1 - c),
  // c = 1 - L; small a as r - (1/L - 3/a) with 1/L - 3/a = -3 S / (a L)
  auto moments = [&](double t, double& F, double& dF) {
    const double a = exp(t);
    double L, C, S, dL;
    langevin_d(a, L, C, S, dL);
    F = a < 0.5 ? r + 3.0 * S / (a * L) : 3.0 / a - C / L - rho;
    dF = a * dL / (L * L) - 3.0 / a;
  };
  double a;
  if (rho < 0.5) {   // a > ~3: psi = e (2 - 3e) / (1 - e), e = 1/a, exact above a = 20
    const double q = 2.0 + rho, disc = q * q - 12.0 * rho;
    a = (q + sqrt(disc > 0.0 ? disc : 0.0)) / (2.0 * rho);
    if (a < 20.0) a = exp(urban_solve(moments, log(a)));
  } else {           // small a: 1/L - 3/a ~ a/5
    a = exp(urban_solve(moments, log(5.0 * r)));
  }
  double L, C, S, dL;
  langevin_d(a, L, C, S, dL);
  const double om = -expm1(-x1);   // 1 - exp(-x1)
  double wi = (om - C) / L;        // 1 - exp(-x1) / L
  if (wi < 0.0) {    // the first moment alone: 1 - L(a) = 1 - exp(-x1)
    auto first = [&](double t, double& F, double& dF) {
      const double aa = exp(t);
      double L1, C1, S1, dL1;
      langevin_d(aa, L1, C1, S1, dL1);
      F = C1 - om;
      dF = -aa * dL1;
    };
    // above a = 20, 1 - L(a) = 1/a exactly
    a = om < 0.05 ? 1.0 / om : exp(urban_solve(first, om < 0.5 ? -log(om) : log(3.0 * (1.0 - om))));
    wi = 0.0;
  }
  if (ua < wi) return 2.0 * (1.0 - ub);
  return -log1p(-(1.0 - ub) * -expm1(-2.0 * a)) / a;
}

// Counts a chunk's electrons per start-of-step tile into census slot q, and
// its electron-steps.  The kKeys keys are the tile's x index mod 16 and its y
// and z indices mod 2, so that sixteen tiles in a row along x (a sparse
// chunk's tiles) or a 2x2 block across y and z (the tiles of an injection
// spot) never share a key.
template <typename T>
__device__ __forceinline__ void chunk_census(const RunDesc& R, ChunkLds<T>& S, uint32_t cell, int q) {
  if (cell != kDead) {
    const int i = cell_i(cell), j = cell_j(cell), k = cell_k(cell);
    const int key = ((i >> 2) & 15) | (((j >> 2) & 1) << 4) | (((k >> 2) & 1) << 5);
    atomicAdd(&S.tc[q][key], 1);
    S.tt[q][key] = tile_of(R, i, j, k);
  }
  const unsigned long long al = __ballot(cell != kDead);
  if ((threadIdx.x & 63) == 0 && al) lds_add(&S.led[L_N + C_ESTEPS], (long long)__popcll(al));
}

// Maximum over the 64 lanes of a wave, in every lane (a scalar): pairs and
// quads, rows of 16 by rotation, then rows 1 and 3 take the last lane of
// the row before and rows 2 and 3 lane 31 (DPP lane moves, no LDS).
__device__ __forceinline__ int wave_max(int x) {
  x = max(x, __builtin_amdgcn_update_dpp(x, x, 0xB1, 0xF, 0xF, false));    // quad_perm [1,0,3,2]
  x = max(x, __builtin_amdgcn_update_dpp(x, x, 0x4E, 0xF, 0xF, false));    // quad_perm [2,3,0,1]
  x = max(x, __builtin_amdgcn_update_dpp(x, x, 0x124, 0xF, 0xF, false));   // row_ror:4
  x = max(x, __builtin_amdgcn_update_dpp(x, x, 0x128, 0xF, 0xF, false));   // row_ror:8
  x = max(x, __builtin_amdgcn_update_dpp(x, x, 0x142, 0xA, 0xF, false));   // row_bcast:15
  x = max(x, __builtin_amdgcn_update_dpp(x, x, 0x143, 0xC, 0xF, false));   // row_bcast:31
  return __builtin_amdgcn_readlane(x, 63);
}

// The regions of a chunk from its census (slot q): each region of the
// previous chunk (tile rt[k], cn holding 5 bits per slot: the chunks it has
// summed) whose tile recurs keeps its slot and its sums, up to the carry
// bound; the most populated other tiles take the free slots.  Returns the
// tiles (nrt), their chunk counts (ncn), the slots carried over (kept) and
// the two fullest tiles (ta, tb).  Tiles sharing a census key pool their
// counts: a worse pick, never a wrong one.  Every wave makes the same picks.
template <typename T>
__device__ __forceinline__ void pick_regions(const ChunkLds<T>& S, int q, const int (&rt)[kRegions], int cn,
                                             int (&nrt)[kRegions], int& ncn, int& kept, int& ta, int& tb) {
  const int l = threadIdx.x & 63;
  const int t = S.tt[q][l];
  int c = t >= 0 ? S.tc[q][l] : 0;
  int a = -1, b = -1, na = 0, nb = 0, m_cn = 0, m_kept = 0;   // fullest two (tile, count)
#pragma unroll
  for (int k = 0; k < kRegions; ++k) {
    nrt[k] = -1;
    const int m = (cn >> (5 * k)) & 31;
    if (rt[k] < 0 || m >= JAcc<T>::max_chunks) continue;
    // a tile has one census key, so at most one lane holds rt[k]
    const unsigned long long mk = __ballot(t == rt[k]);
    const int cc = mk ? __builtin_amdgcn_readlane(c, __ffsll((long long)mk) - 1) : 0;
    if (cc == 0) continue;
    nrt[k] = rt[k];
    m_cn |= (m + 1) << (5 * k);
    m_kept |= 1 << k;
    if (cc > na) { b = a; nb = na; a = rt[k]; na = cc; }
    else if (cc > nb) { b = rt[k]; nb = cc; }
    if (t == rt[k]) c = 0;
  }
  bool more = true;   // tiles left to place (no early exit: every slot index stays static)
#pragma unroll
  for (int k = 0; k < kRegions; ++k) {
    if (!more || nrt[k] >= 0) continue;
    const int key = wave_max(c > 0 ? (c << 6) | l : -1);
    if (key < 0) { more = false; continue; }
    const int tile = __builtin_amdgcn_readlane(t, key & 63);
    if (tile < 0) { more = false; continue; }   // (a counted key always names its tile)
    const int cnt = key >> 6;
    nrt[k] = tile;
    m_cn |= 1 << (5 * k);
    if (cnt > na) { b = a; nb = na; a = tile; na = cnt; }
    else if (cnt > nb) { b = tile; nb = cnt; }
    if (l == (key & 63)) c = 0;
  }
  ncn = m_cn;
  kept = m_kept;
  ta = a;
  tb = b;
}

// The first thread claims, for this step, the tile of every slot that took
// a new tile for this chunk (bit k of fresh; the carried regions keep their
// claim), and records in S.own whether this workgroup was the first.  The
// atomics go out after the chunk's state loads, which the wave waits for
// next anyway.
template <typename T>
__device__ __forceinline__ void claim_regions(const RunDesc& R, ChunkLds<T>& S, const int (&rt)[kRegions],
                                              int fresh, int stampv) {
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kRegions; ++k)
      if ((fresh >> k) & 1) S.own[k] = atomicMax(&R.tstamp[rt[k]], stampv) < stampv;
  }
}

// ---------------------------------------------------------------------------
// the particle step: gather, Boris, deposit, move, ionisation,
// bremsstrahlung, elastic scatter, boundaries, low-energy removal
// ---------------------------------------------------------------------------
// Waves per SIMD the register allocation of the particle kernel is held to.
// The kernel is latency bound (dependent HBM round trips per chunk), so
// occupancy pays for a few spills: 2 in FP64 (256 registers), 4 in FP32.
template <typename T> struct PartOcc { static constexpr int waves = 2; };
template <> struct PartOcc<float> { static constexpr int waves = 4; };
// Variants (V, bits): delta rays (own optical depth, spawning); the
// Urban-type scatter.  Each adds registers that the plain step need not hold.
enum : int { kVarDelta = 1, kVarUrban = 2 };
template <typename T, int V>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(PartOcc<T>::waves))) void k_particle(const RunDesc* __restrict__ runs,
                                                     const BlockMap* __restrict__ bmap) {
  constexpr bool D = (V & kVarDelta) != 0;
  constexpr bool UR = (V & kVarUrban) != 0;
  const BlockMap bm = bmap[blockIdx.x];
  if (bm.nb < 8) return;   // alignment padding between runs
  const RunDesc& R = runs[bm.run];
  const auto ctr = G(R.ctr);
  if (!ctr->active) return;
  const long long step = ctr->step;
  long long n = ctr->n_total + inject_count(R, step);
  n = n < R.capacity ? n : R.capacity;
  const PartG<T> P = part_g<T>(R.p[ctr->cur]);
  const bool count = sort_step(R.sort_every, step);
  __shared__ ChunkLds<T> S;
  long long acc[L_N];   // ledger terms; event counts and rare terms go to S.led
#pragma unroll
  for (int i = 0; i < L_N; ++i) acc[i] = 0;

  const int nx = R.nx, ny = R.ny, nz = R.nz;
  const int sx = nx + 1, sxy = (nx + 1) * (ny + 1);
  const uint32_t phys = R.physics;
  const gptr<const T> E0 = G((const T*)R.E[0]), E1 = G((const T*)R.E[1]), E2 = G((const T*)R.E[2]);
  const gptr<const T> B0 = G((const T*)R.B[0]), B1 = G((const T*)R.B[1]), B2 = G((const T*)R.B[2]);
  TableView<T> tab{G((const T*)R.tab_X), G((const T*)R.tab_SIG), G((const T*)R.tab_SUB), R.tab_nT, R.tab_nr,
                   (T)R.tab_ln_kcut, (T)R.tab_s_scale, (T)R.tab_kcut};
  const T e_kick = (T)R.e_kick, b_rot = (T)R.b_rot, cdt = (T)R.cdt_dx;
  const T ledS = (T)kLedScale;


  const ChunkRange cr = chunk_run(bm, n);
  lds_init(S);
  const bool lds_tab = R.tab_nT <= kLdsTab;
  if (lds_tab)
    for (int t = threadIdx.x; t < R.tab_nT; t += kBlock) {
      S.tsig[t] = tab.SIG[t];
      S.tsub[t] = tab.SUB[t];
    }
  __syncthreads();
  uint32_t cell_next = kDead;   // packed cell of this thread's electron in the next chunk
  if (cr.beg < cr.end && cr.beg * kBlock + threadIdx.x < n) cell_next = P.cell[cr.beg * kBlock + threadIdx.x];
  // tile offsets returned by the counting atomics, stored a chunk later
  unsigned base_val = 0, far_val = 0;
  long long base_at = -1, far_at = -1;
  int f_tile0 = -1, f_tile1 = -1;       // tiles whose field halos the two LDS slots hold
  // The regions: the chunk's most populated tiles, up to kRegions, each with
  // an LDS slot for its electrons' current and heat.  A chunk of tile-sorted
  // electrons spans one tile where ~200 electrons share a tile and several
  // where few do (3 at the median, 7 at the 90th percentile at ~55 per
  // tile); the newly injected electrons at the buffer's tail are not yet
  // sorted and spread over the tiles of the injection spot.  The regions of
  // the next chunk are picked at the end of this one, from the cells already
  // prefetched, so that regions whose tile continues keep their sums and the
  // others are flushed while the next chunk's state is in flight.
  int rt[kRegions], fl[kRegions];   // tile of each slot now; tile to flush from each slot (-1 none)
  int cn = 0, ta = -1, tb = -1;     // chunk counts per slot; the two fullest tiles
  int pta = -1;                     // fullest tile of the previous chunk (its destination bins)
  constexpr bool kFlushEarly = sizeof(T) == 8;
  long long pch = -1;               // the previous chunk
#pragma unroll
  for (int k = 0; k < kRegions; ++k) { rt[k] = -1; fl[k] = -1; }
  const int stampv = (int)(step + 1);
  int fresh = 0;                    // slots that took a new tile for the coming chunk
  if (cr.beg < cr.end) {
    chunk_census(R, S, cell_next, 0);
    __syncthreads();
    int nrt[kRegions], kept;
    pick_regions<T>(S, 0, rt, 0, nrt, cn, kept, ta, tb);
#pragma unroll
    for (int k = 0; k < kRegions; ++k) {
      rt[k] = nrt[k];
      if (rt[k] >= 0) fresh |= 1 << k;
    }
  }
  int slot = 0;
  for (long long ch = cr.beg; ch < cr.end; ch += cr.stride, slot ^= 1) {
    const long long i = ch * kBlock + threadIdx.x;
    const uint32_t cell = cell_next;
    {
      const long long in = (ch + cr.stride) * kBlock + threadIdx.x;
      cell_next = ch + cr.stride < cr.end && in < n ? P.cell[in] : kDead;
    }
    int ci = 0, cj = 0, ck = 0, my_tile = -1;
    // the electron's state is in flight while the previous chunk's regions are flushed
    T ox = 0, oy = 0, oz = 0, ux = 0, uy = 0, uz = 0, wn = 0, tau = 0, taud = 0;
    uint32_t id = 0;
    if (cell != kDead) {
      ci = cell_i(cell); cj = cell_j(cell); ck = cell_k(cell);
      my_tile = tile_of(R, ci, cj, ck);
      // FP32: one load per field (a compiler barrier between them stops the
      // merge into dwordx4 loads, whose register tuples cost spills here:
      // 2.029 -> 2.010 ms per step); FP64 keeps the merged loads
      constexpr bool kSplit = sizeof(T) == 4;
      ox = P.ox[i];
      if constexpr (kSplit) asm volatile("" ::: "memory");
      oy = P.oy[i];
      if constexpr (kSplit) asm volatile("" ::: "memory");
      oz = P.oz[i];
      if constexpr (kSplit) asm volatile("" ::: "memory");
      ux = P.ux[i];
      if constexpr (kSplit) asm volatile("" ::: "memory");
      uy = P.uy[i];
      if constexpr (kSplit) asm volatile("" ::: "memory");
      uz = P.uz[i];
      if constexpr (kSplit) asm volatile("" ::: "memory");
      wn = P.wn[i];
      if constexpr (kSplit) asm volatile("" ::: "memory");
      tau = P.tau[i];
      id = P.id[i];
      if constexpr (D) {   // a batch may mix runs with and without delta rays
        if (phys & PHYS_DELTA) taud = P.taud[i];
      }
    }
    // the previous chunk's regions that do not carry over, and its
    // destination counts, go to HBM while this chunk's state is in flight
    // (FP64 flushed them at the previous chunk's end: it has no registers to
    // spare for the state loads in flight)
    if (!kFlushEarly && pch >= 0) {
#pragma unroll
      for (int k = 0; k < kRegions; ++k)
        if (fl[k] >= 0) lds_flush_region(R, S, k, fl[k], stampv);
      if (count) lds_flush_counts(R, S, make_home(R, pta), pch, base_val, base_at);
    }
    __syncthreads();
    // this chunk's census was read when its regions were picked; the
    // previous regions of reused slots are flushed
    if (threadIdx.x < kKeys) { S.tc[slot][threadIdx.x] = 0; S.tt[slot][threadIdx.x] = -1; }
    claim_regions(R, S, rt, fresh, stampv);
    const Home hm = make_home(R, ta), hm2 = make_home(R, tb);
    if (phys & PHYS_FIELDS) {
      // a region whose halo a slot already holds keeps it (fields do not
      // change during the launch); a new one takes the other region's free
      // slot, else the slot of the smaller (older) tile
      int fs_a = !hm.ok ? -1 : (f_tile0 == ta ? 0 : (f_tile1 == ta ? 1 : -1));
      int fs_b = !hm2.ok ? -1 : (f_tile0 == tb ? 0 : (f_tile1 == tb ? 1 : -1));
      const bool need_a = hm.ok && fs_a < 0;
      if (need_a) fs_a = fs_b >= 0 ? 1 - fs_b : (f_tile0 <= f_tile1 ? 0 : 1);
      const bool need_b = hm2.ok && fs_b < 0;
      if (need_b) fs_b = 1 - fs_a;
      const int nst = (need_a ? 1 : 0) + (need_b ? 1 : 0);
      if (nst) {
        // the new halos, staged in LDS: the six field loads of a node are
        // issued together (rows of 6 nodes along x are contiguous in HBM);
        // nodes outside the grid are never gathered
#pragma unroll 1
        for (int t = threadIdx.x; t < nst * kHaloN; t += kBlock) {
          const bool is_a = need_a && t < kHaloN;
          const int l = t >= kHaloN ? t - kHaloN : t;
          const int i = (is_a ? hm.bx : hm2.bx) + l % kHalo;
          const int j = (is_a ? hm.by : hm2.by) + (l / kHalo) % kHalo;
          const int k = (is_a ? hm.bz : hm2.bz) + l / (kHalo * kHalo);
          const bool in = i >= 0 && j >= 0 && k >= 0 && i <= nx && j <= ny && k <= nz;
          const long long o = in ? i + (long long)sx * j + (long long)sxy * k : 0;
          T v[6];
          v[0] = in ? E0[o] : (T)0;
          v[1] = in ? E1[o] : (T)0;
          v[2] = in ? E2[o] : (T)0;
          v[3] = in ? B0[o] : (T)0;
          v[4] = in ? B1[o] : (T)0;
          v[5] = in ? B2[o] : (T)0;
          T* d = &S.F[is_a ? fs_a : fs_b][0][l];
#pragma unroll
          for (int f = 0; f < 6; ++f) d[f * kHaloN] = v[f];
        }
        if (need_a) { if (fs_a == 0) f_tile0 = ta; else f_tile1 = ta; }
        if (need_b) { if (fs_b == 0) f_tile0 = tb; else f_tile1 = tb; }
        __syncthreads();
      }
    }
    // offsets returned by the previous chunk's atomics: waiting for them here
    // costs nothing, this chunk's loads (issued later) have landed
    if (base_at >= 0) { G(R.chunk_base)[base_at] = base_val; base_at = -1; }
    if (far_at >= 0) { G(R.far_off)[far_at] = far_val; far_at = -1; }
    int dest_bin = -1;
    if (cell != kDead) {
      // LDS slot of the electron's tile (-1: none), the first node of that
      // tile's halo, and the staged field halo of the tile (-1: none)
      int js = -1;
#pragma unroll
      for (int k = 0; k < kRegions; ++k) js = my_tile == rt[k] ? k : js;
      // no LDS region: its current and heat go to the accumulators, and the
      // tile is marked for the gather
      if (js < 0) G(R.tdirty)[my_tile] = stampv;
      const int rbx = (ci & ~(kTile - 1)) - 1, rby = (cj & ~(kTile - 1)) - 1, rbz = (ck & ~(kTile - 1)) - 1;
      const int fsl = my_tile == f_tile0 ? 0 : (my_tile == f_tile1 ? 1 : -1);
      typename JAcc<T>::type* Js = js >= 0 ? S.J[js] : nullptr;
      const int heat_cell = ci + nx * (cj + ny * ck);
      const int heat_local = (ci & 3) + 4 * (cj & 3) + 16 * (ck & 3);

      T u2 = ux * ux + uy * uy + uz * uz;
      const T eps0 = kinetic(u2, m_sqrt((T)1 + u2));

      // stencils at x^n (shared by gather and deposit)
      const Axis<T> nxa = node_axis(ci, ox), nya = node_axis(cj, oy), nza = node_axis(ck, oz);
      const Axis<T> sxa = stag_axis(ci, ox, nx), sya = stag_axis(cj, oy, ny), sza = stag_axis(ck, oz, nz);

      // --- gather + Boris push (q = -e) ---
      if (phys & PHYS_FIELDS) {
        T Ex, Ey, Ez, Bx, By, Bz;
        if (fsl >= 0) {   // from a halo staged in LDS
          const T* F = &S.F[fsl][0][0];
          Ex = gather8_lds(F, rbx, rby, rbz, sxa, nya, nza);
          Ey = gather8_lds(F + kHaloN, rbx, rby, rbz, nxa, sya, nza);
          Ez = gather8_lds(F + 2 * kHaloN, rbx, rby, rbz, nxa, nya, sza);
          Bx = gather8_lds(F + 3 * kHaloN, rbx, rby, rbz, nxa, sya, sza);
          By = gather8_lds(F + 4 * kHaloN, rbx, rby, rbz, sxa, nya, sza);
          Bz = gather8_lds(F + 5 * kHaloN, rbx, rby, rbz, sxa, sya, nza);
        } else {
          Ex = gather8(E0, sx, sxy, sxa, nya, nza);
          Ey = gather8(E1, sx, sxy, nxa, sya, nza);
          Ez = gather8(E2, sx, sxy, nxa, nya, sza);
          Bx = gather8(B0, sx, sxy, nxa, sya, sza);
          By = gather8(B1, sx, sxy, sxa, nya, sza);
          Bz = gather8(B2, sx, sxy, sxa, sya, nza);
        }
        const T ex = e_kick * Ex, ey = e_kick * Ey, ez = e_kick * Ez;
        const T mx = ux + ex, my = uy + ey, mz = uz + ez;
        const T gi = b_rot / m_sqrt((T)1 + mx * mx + my * my + mz * mz);
        const T tx = gi * Bx, ty = gi * By, tz = gi * Bz;
        const T sf = (T)2 / ((T)1 + tx * tx + ty * ty + tz * tz);
        const T sxv = sf * tx, syv = sf * ty, szv = sf * tz;
        const T px = mx + (my * tz - mz * ty), py = my + (mz * tx - mx * tz), pz = mz + (mx * ty - my * tx);
        ux = mx + (py * szv - pz * syv) + ex;
        uy = my + (pz * sxv - px * szv) + ey;
        uz = mz + (px * syv - py * sxv) + ez;
      }
      u2 = ux * ux + uy * uy + uz * uz;
      T g = m_sqrt((T)1 + u2);
      const T eps1 = kinetic(u2, g);
      {
        const T dW = eps1 - eps0;
        if (dW > (T)0) acc[L_FIELD_GAIN] += to_fixed(dW * wn * ledS);
        else acc[L_FIELD_LOSS] += to_fixed(-dW * wn * ledS);
      }
      const T ig = (T)1 / g;
      const T vx = ux * ig, vy = uy * ig, vz = uz * ig;

      // --- hot-current deposit at x^n with the pushed velocity ---
      {
        const T amp = -wn * (T)(kJScale / (double)(1LL << JAcc<T>::shift));
        constexpr int CN = kHaloN;
        deposit8(R.Jacc[0], Js, rbx, rby, rbz, sx, sxy, sxa, nya, nza, amp * vx);
        deposit8(R.Jacc[1], Js ? Js + CN : Js, rbx, rby, rbz, sx, sxy, nxa, sya, nza, amp * vy);
        deposit8(R.Jacc[2], Js ? Js + 2 * CN : Js, rbx, rby, rbz, sx, sxy, nxa, nya, sza, amp * vz);
      }

      // --- move ---
      ox += vx * cdt; oy += vy * cdt; oz += vz * cdt;
      {
        const T fx = m_floor(ox), fy = m_floor(oy), fz = m_floor(oz);
        ci += (int)fx; cj += (int)fy; ck += (int)fz;
        ox -= fx; oy -= fy; oz -= fz;
      }

      // --- ionisation, eq. (stop_ion); with delta rays the restricted loss ---
      T eps2 = eps1;
      long long heat = 0;
      if ((phys & PHYS_ION) && u2 > (T)0) {
        T dE;
        if (D && (phys & PHYS_DELTA)) {
          dE = restricted_loss(R, eps1, g, u2);
        } else {
          const T beta = m_sqrt(u2) * ig;
          // ln(eps) + ln(g + 1) / 2 as one logarithm
          T L = (T)0.5 * m_log(eps1 * eps1 * (g + (T)1)) - (T)R.ln_iex + (T)0.909 * ig * ig - (T)0.818 * ig - (T)0.246;
          L = L > (T)0 ? L : (T)0;
          dE = (T)R.c_ion * L / beta;
        }
        dE = dE < eps1 ? dE : eps1;
        const T sc = umag_of(eps1 - dE) / m_sqrt(u2);
        ux *= sc; uy *= sc; uz *= sc;
        u2 = ux * ux + uy * uy + uz * uz;
        g = m_sqrt((T)1 + u2);
        eps2 = kinetic(u2, g);
        const T ion = (eps1 - eps2) * wn;
        acc[L_ION] += to_fixed(ion * ledS);
        heat += to_fixed(ion * (T)kHeatScale);
      }

      // --- delta rays: Moller scatter above the cut, own optical depth, one
      // per step at most; born at x^n with the parent's weight ---
      if constexpr (D) {
        if ((phys & PHYS_DELTA) && u2 > (T)0) {
          const T dcut = (T)R.d_cut;
          const bool open = eps2 > (T)2 * dcut;
          const T gi2 = (T)1 / (g * g);
          const T a = ((T)2 * g - (T)1) * gi2, b = eps2 * eps2 * gi2;
          const T xc = dcut / eps2;
          if (open) {
            const T J = b * ((T)0.5 - xc) + (T)1 / xc - (T)1 / ((T)1 - xc) - a * m_log(((T)1 - xc) / xc);
            taud -= (T)R.k_mol * J * g / (m_sqrt(u2) * eps2);
          }
          if (open && taud < (T)0) {
            // energy fraction by rejection from 1/x^2 on [x_c, 1/2]
            const T gmax = fmax(moller_g(xc, a, b), moller_g((T)0.5, a, b));
            const T span = (T)1 - (T)2 * xc;
            T x = xc;
#pragma unroll 1
            for (int k = 0; k < kDeltaTries / 2; ++k) {
              const Uni4<T> u = draws<T>(id, R.seed, step, SLOT_DELTA_TRY + k);
              const T c0 = xc / ((T)1 - u.a * span);
              if (u.b * gmax <= moller_g(c0, a, b)) { x = c0; break; }
              x = xc / ((T)1 - u.c * span);   // kept if accepted or if it is the last candidate
              if (u.d * gmax <= moller_g(x, a, b)) break;
            }
            const T ed = x * eps2;
            const Uni4<T> uk = draws<T>(id, R.seed, step, SLOT_DELTA_K);
            // two-body kinematics on a free electron at rest
            T cth = m_sqrt(ed * (eps2 + (T)2) / (eps2 * (ed + (T)2)));
            cth = cth < (T)1 ? cth : (T)1;
            const T um = m_sqrt(u2);
            T dx_ = ux, dy_ = uy, dz_ = uz;
            rotate(dx_, dy_, dz_, m_acos(cth), uk.a);
            const T sd = umag_of(ed) / um;
            dx_ *= sd; dy_ *= sd; dz_ *= sd;
            T qx = ux - dx_, qy = uy - dy_, qz = uz - dz_;
            const T sq = umag_of(eps2 - ed) / m_sqrt(qx * qx + qy * qy + qz * qz);
            ux = qx * sq; uy = qy * sq; uz = qz * sq;
            taud = -m_log((T)1 - uk.b);
            u2 = ux * ux + uy * uy + uz * uz;
            g = m_sqrt((T)1 + u2);
            const T eps_p = kinetic(u2, g);
            lds_add(&S.led[L_N + C_DELTA], 1LL);
            T resid = eps2 - eps_p - ed;
            bool local = ed < (T)R.e_min;
            if (!local) {
              // record slots: one atomic per wave on the run's counter (the
              // lanes here are the wave's spawning electrons)
              const int lane = threadIdx.x & 63;
              const unsigned long long act = __ballot(1);
              const int lead = __ffsll((long long)act) - 1;
              unsigned long long base = 0;
              if (lane == lead)
                base = __hip_atomic_fetch_add((__attribute__((address_space(1))) unsigned long long*)&ctr->n_spawn,
                                              (unsigned long long)__popcll(act), __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
              base = ((unsigned long long)(unsigned)__shfl((int)(base >> 32), lead, 64) << 32) |
                     (unsigned)__shfl((int)(unsigned)base, lead, 64);
              const unsigned long long a_ = base + (unsigned long long)__popcll(act & ((1ull << lane) - 1ull));
              if ((long long)a_ < R.spawn_cap) {
                // the record: birth place x^n (still in this electron's slot)
                G(R.sp_cell)[a_] = cell;
                G(R.sp_pid)[a_] = id;
                G((T*)R.sp_f[0])[a_] = P.ox[i];
                G((T*)R.sp_f[1])[a_] = P.oy[i];
                G((T*)R.sp_f[2])[a_] = P.oz[i];
                G((T*)R.sp_f[3])[a_] = dx_;
                G((T*)R.sp_f[4])[a_] = dy_;
                G((T*)R.sp_f[5])[a_] = dz_;
                G((T*)R.sp_f[6])[a_] = wn;
                // birth-tile counts: one atomic per distinct tile of the wave's records
                unsigned long long todo = __ballot(1);
                while (todo) {
                  const int l2 = __ffsll((long long)todo) - 1;
                  const int t2 = __shfl(my_tile, l2, 64);
                  const unsigned long long m = __ballot(my_tile == t2) & todo;
                  if (lane == l2) atomic_add_u32(&R.sp_cnt[t2], (unsigned)__popcll(m));
                  todo &= ~m;
                }
                const T d2 = dx_ * dx_ + dy_ * dy_ + dz_ * dz_;
                resid += ed - kinetic(d2, m_sqrt((T)1 + d2));
              } else {
                local = true;
                lds_add(&S.led[L_N + C_DELTA_LOST], 1LL);
              }
            }
            if (local) {   // stops where it is born
              lds_add(&S.led[L_STOPPED], to_fixed(ed * wn * ledS));
              heat += to_fixed(ed * wn * (T)kHeatScale);
            }
            lds_add(&S.led[L_RESIDUAL], to_fixed(resid * wn * ledS));
            eps2 = eps_p;
          }
        }
      }

      // --- bremsstrahlung: optical depth, one emission per step at most ---
      Uni4<T> cd{};
      if (phys & (PHYS_BREM | PHYS_SCATTER)) cd = draws<T>(id, R.seed, step, SLOT_COLLIDE);
      T eps3 = eps2;
      bool emitted = false;
      if ((phys & PHYS_BREM) && u2 > (T)0) {
        const T lne = m_log(eps2);
        int tj;
        T tf;
        tab.row(lne, tj, tf);
        const bool above = eps2 > tab.kcut;   // no emission at or below k_cut
        // the inverse-CDF exponent of a possible emission is fetched together
        // with the cross sections, so one memory round trip serves both
        const T xs = above ? tab.x_at(tj, tf, cd.d) : (T)0;
        T sg0, sg1, sb0, sb1;
        if (lds_tab) {
          sg0 = S.tsig[tj]; sg1 = S.tsig[tj + 1]; sb0 = S.tsub[tj]; sb1 = S.tsub[tj + 1];
        } else {
          sg0 = tab.SIG[tj]; sg1 = tab.SIG[tj + 1]; sb0 = tab.SUB[tj]; sb1 = tab.SUB[tj + 1];
        }
        const T um = m_sqrt(u2);
        const T beta = um / g;
        // cross-sections of the start-of-step cell, optionally times eq. F_sigma
        const T fs = (phys & PHYS_FSIGMA) ? G((const T*)R.fsig)[heat_cell] : (T)1;
        tau -= (T)R.k_brem * fs * (above ? sg0 + tf * (sg1 - sg0) : (T)0) * beta;
        const T sub = (T)R.k_sub * fs * (above ? sb0 + tf * (sb1 - sb0) : eps2) * beta;
        T kph = (T)0;
        if (tau < (T)0) {
          kph = tab.kcut * m_exp(xs * (lne - tab.ln_kcut));
          // the optical depth is redrawn with the photon's tally below
          // the photon's tally waits in LDS for the end of this electron's step
          const int t = threadIdx.x;
          S.ph[0][t] = kph; S.ph[1][t] = ux; S.ph[2][t] = uy; S.ph[3][t] = uz; S.ph[4][t] = um; S.ph[5][t] = g;
          emitted = true;
        }
        const T kb = kph * (T)R.inv_boost;
        const T room = eps2 - kb;                   // >= 0: k <= eps2, boost >= 1
        const T sub_a = sub < room ? sub : room;    // sub-cut loss actually applied
        const T sc = umag_of(room - sub_a) / um;
        ux *= sc; uy *= sc; uz *= sc;
        u2 = ux * ux + uy * uy + uz * uz;
        g = m_sqrt((T)1 + u2);
        eps3 = kinetic(u2, g);
        acc[L_RAD_S] += to_fixed(sub_a * wn * ledS);
        acc[L_RESIDUAL] += to_fixed((eps2 - eps3 - kb - sub_a) * wn * ledS);
      }

      // --- elastic scatter: Davies, or the Urban-type model functions ---
      if ((phys & PHYS_SCATTER) && u2 > (T)0) {
        if (UR && (phys & PHYS_URBAN)) {
          const double w = urban_one_minus_cos(R, (double)u2, (double)cd.a, (double)cd.b);
          rotate_cs(ux, uy, uz, (T)(1.0 - w), (T)sqrt(w * (2.0 - w)), cd.c);
        } else {
          const T um = m_sqrt(u2);
          const T iu = (T)1 / um;
          T lg = m_log((T)R.l_dav * um);
          lg = lg > (T)0 ? lg : (T)0;
          const T s2 = (T)R.c_dav * g * (iu * iu * iu) * lg;
          T sb, cb;
          m_sincos2pi(cd.b, sb, cb);
          const T gam = m_sqrt((T)-2 * m_log(cd.a)) * cb;
          T sn, cs;
          m_sincos(gam * m_sqrt(s2), sn, cs);
          rotate_known(ux, uy, uz, um, iu, cs, sn, cd.c);
        }
        // elastic: any change of the stored energy is rounding, booked apart
        u2 = ux * ux + uy * uy + uz * uz;
        g = m_sqrt((T)1 + u2);
        const T eps_r = kinetic(u2, g);
        acc[L_RESIDUAL] += to_fixed((eps3 - eps_r) * wn * ledS);
        eps3 = eps_r;
      }

      // --- boundaries: x (slab faces), y, z (domain walls) ---
      T eps = eps3;
      bool alive = true;
      {
        // one copy of the boundary code for the three axes: (c0, o0) is the
        // axis being checked, and the triples rotate by one per axis
        int c0 = ci, c1 = cj, c2 = ck;
        T o0 = ox, o1 = oy, o2 = oz;
#pragma unroll 1
        for (int a = 0; a < 3; ++a) {
          const int lo = a == 0 ? R.ix_lo : 0, hi = a == 0 ? R.ix_hi : (a == 1 ? ny : nz);
          if (alive) alive = boundary_axis(R, a, c0, o0, lo, hi, ux, uy, uz, eps, wn, id, step, S.led);
          const int ct = c0; c0 = c1; c1 = c2; c2 = ct;
          const T ot = o0; o0 = o1; o1 = o2; o2 = ot;
        }
        ci = c0; cj = c1; ck = c2;
        ox = o0; oy = o1; oz = o2;
      }

      // --- removal below e_min, energy to the cell's heat ---
      if (alive && eps < (T)R.e_min) {
        lds_add(&S.led[L_STOPPED], to_fixed(eps * wn * ledS));
        lds_add(&S.led[L_N + C_STOPPED], 1LL);
        heat += to_fixed(eps * wn * (T)kHeatScale);
        alive = false;
      }
      if (heat != 0) {
        if (js >= 0)
          lds_add(&S.heat[js][heat_local], heat);
        else atomic_add_i64(&R.heat_acc[heat_cell], heat);
      }
      if (!alive) {
        P.cell[i] = kDead;
      } else {
        // the whole record, unchanged fields too: whole lines reach HBM
        // without a read-modify-write of the parts left out
        P.cell[i] = pack_cell(ci, cj, ck);
        P.id[i] = id;
        P.ox[i] = ox; P.oy[i] = oy; P.oz[i] = oz;
        P.ux[i] = ux; P.uy[i] = uy; P.uz[i] = uz;
        P.wn[i] = wn;
        P.tau[i] = tau;
        if constexpr (D) {
          if (phys & PHYS_DELTA) P.taud[i] = taud;
        }
        if (count) {   // destination tile for the sort that ends this step
          const int tx = ci >> 2, ty = cj >> 2, tz = ck >> 2;
          dest_bin = nb_bin(hm, tx, ty, tz);
          if (dest_bin < 0) {
            far_val = atomic_add_u32(&R.tile_cnt[tx + R.ntx * (ty + R.nty * tz)], 1u);
            far_at = i;
          }
        }
      }
      if (emitted) {
        // emission is rare: its tally runs here, where little of the
        // electron's state is still live; the empty asm keeps the compiler
        // from carrying the queued values in registers instead of LDS
        asm volatile("" ::: "memory");
        const T tau_new = photon_tally(R, S, wn, id, step);
        if (alive) P.tau[i] = tau_new;
      }
    }
    if (count) {
      // most electrons of a chunk land in one tile: count it with one atomic
      // per wave, the rest one by one
      const int lead = __builtin_amdgcn_readlane(dest_bin, 0);
      const unsigned long long same = __ballot(dest_bin == lead && dest_bin >= 0);
      if ((threadIdx.x & 63) == 0 && same) atomicAdd(&S.cnt[lead], (unsigned)__popcll(same));
      if (dest_bin >= 0 && dest_bin != lead) atomicAdd(&S.cnt[dest_bin], 1u);
    }
    if (count && threadIdx.x == 0) G(R.chunk_home)[ch] = hm.ok ? ta : kNoTile;
    // the next chunk's census and regions
    chunk_census(R, S, cell_next, slot ^ 1);
    __syncthreads();
    {
      int nrt[kRegions], ncn, kept, nta, ntb;
      pick_regions<T>(S, slot ^ 1, rt, cn, nrt, ncn, kept, nta, ntb);
      fresh = 0;
#pragma unroll
      for (int k = 0; k < kRegions; ++k) {
        if (nrt[k] >= 0 && !((kept >> k) & 1)) fresh |= 1 << k;
        fl[k] = rt[k] >= 0 && !((kept >> k) & 1) ? rt[k] : -1;
        rt[k] = nrt[k];
      }
      cn = ncn;
      pta = ta; ta = nta; tb = ntb;
      pch = ch;
    }
    if (kFlushEarly) {
#pragma unroll
      for (int k = 0; k < kRegions; ++k)
        if (fl[k] >= 0) lds_flush_region(R, S, k, fl[k], stampv);
      if (count) lds_flush_counts(R, S, make_home(R, pta), pch, base_val, base_at);
    }
  }
  // the last chunk's regions and destination counts
  if (!kFlushEarly && pch >= 0) {
#pragma unroll
    for (int k = 0; k < kRegions; ++k)
      if (fl[k] >= 0) lds_flush_region(R, S, k, fl[k], stampv);
    if (count) lds_flush_counts(R, S, make_home(R, pta), pch, base_val, base_at);
  }
  if (base_at >= 0) G(R.chunk_base)[base_at] = base_val;
  if (far_at >= 0) G(R.far_off)[far_at] = far_val;
  block_flush<L_N, 0, L_N + C_N>(acc, R.acc_led, R.events, S.led);
}

// ---------------------------------------------------------------------------
// tile sort: scan of the destination counts, then scatter of the electrons
// into the other particle buffer in tile order (dead electrons dropped).
// The same three scan kernels also number the step's delta rays by birth
// tile (which = 1).
// ---------------------------------------------------------------------------
struct ScanSet { gptr<unsigned> cnt, start, blk; bool on; };

__device__ __forceinline__ ScanSet scan_set(const RunDesc& R, int which) {
  const auto ctr = G(R.ctr);
  if (which == 0)
    return ScanSet{G(R.tile_cnt), G(R.tile_start), G(R.scan_blk),
                   ctr->active && sort_step(R.sort_every, ctr->step)};
  return ScanSet{G(R.sp_cnt), G(R.sp_start), G(R.sp_blk), ctr->active && (R.physics & PHYS_DELTA) != 0};
}

__global__ __launch_bounds__(kBlock) void k_scan_reduce(const RunDesc* __restrict__ runs,
                                                        const BlockMap* __restrict__ bmap, int which) {
  const BlockMap bm = bmap[blockIdx.x];
  const RunDesc& R = runs[bm.run];
  const ScanSet Q = scan_set(R, which);
  if (!Q.on) return;
  __shared__ unsigned sm[kBlock];
  const int t0 = bm.lb * kScanTile;
  unsigned s = 0;
  for (int t = t0 + threadIdx.x; t < t0 + kScanTile && t < R.ntiles; t += kBlock) s += Q.cnt[t];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) Q.blk[bm.lb] = sm[0];
}

// exclusive scan of the block sums (one workgroup per run)
__global__ __launch_bounds__(kBlock) void k_scan_blocks(const RunDesc* __restrict__ runs,
                                                        const BlockMap* __restrict__ bmap, int which) {
  const BlockMap bm = bmap[blockIdx.x];
  const RunDesc& R = runs[bm.run];
  const ScanSet Q = scan_set(R, which);
  if (!Q.on) return;
  __shared__ unsigned sm[kBlock];
  __shared__ unsigned carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < R.scan_nblk; base += kBlock) {
    const int t = base + threadIdx.x;
    const unsigned v = t < R.scan_nblk ? Q.blk[t] : 0u;
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < kBlock; o <<= 1) {   // inclusive Hillis-Steele scan
      const unsigned a = threadIdx.x >= o ? sm[threadIdx.x - o] : 0u;
      __syncthreads();
      sm[threadIdx.x] += a;
      __syncthreads();
    }
    if (t < R.scan_nblk) Q.blk[t] = carry + sm[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == kBlock - 1) carry += sm[kBlock - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0 && which == 0) G(R.ctr)->n_sorted = carry;
}

// tile starts and scatter cursors
__global__ __launch_bounds__(kBlock) void k_scan_tiles(const RunDesc* __restrict__ runs,
                                                       const BlockMap* __restrict__ bmap, int which) {
  const BlockMap bm = bmap[blockIdx.x];
  const RunDesc& R = runs[bm.run];
  const ScanSet Q = scan_set(R, which);
  if (!Q.on) return;
  __shared__ unsigned sm[kBlock];
  constexpr int per = kScanTile / kBlock;   // tiles per thread
  const int t0 = bm.lb * kScanTile + threadIdx.x * per;
  unsigned v[per];
  unsigned s = 0;
#pragma unroll
  for (int q = 0; q < per; ++q) {
    v[q] = t0 + q < R.ntiles ? Q.cnt[t0 + q] : 0u;
    s += v[q];
  }
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < kBlock; o <<= 1) {
    const unsigned a = threadIdx.x >= o ? sm[threadIdx.x - o] : 0u;
    __syncthreads();
    sm[threadIdx.x] += a;
    __syncthreads();
  }
  unsigned run = Q.blk[bm.lb] + sm[threadIdx.x] - s;
#pragma unroll
  for (int q = 0; q < per; ++q) {
    if (t0 + q < R.ntiles) Q.start[t0 + q] = run;
    run += v[q];
  }
}

// Scatter of the electrons into the other particle buffer in tile order
// (dead electrons dropped).  The particle kernel fixed where each chunk's
// electrons bound for a tile go (tile start + the chunk's offset in it); here
// each chunk ranks its electrons inside their destination bins, gathers them
// in LDS in bin order, and writes every bin's run with consecutive threads,
// so that a run reaches HBM as whole sectors rather than one piece per wave.
// Electrons bound outside the chunk's bins (rare) are written directly.
template <typename T> struct ScatterLds {
  unsigned cnt[kNbN];          // electrons per bin, then (after the scan) bin starts
  unsigned start[kNbN];
  T f[9][kBlock];              // ox oy oz ux uy uz wn tau taud, in bin order
  uint32_t cell[kBlock], id[kBlock];
  unsigned char bin[kBlock];
};

template <typename T, bool D>
__global__ __launch_bounds__(kBlock) void k_scatter(const RunDesc* __restrict__ runs,
                                                    const BlockMap* __restrict__ bmap) {
  const BlockMap bm = bmap[blockIdx.x];
  if (bm.nb < 8) return;
  const RunDesc& R = runs[bm.run];
  const auto ctr = G(R.ctr);
  if (!ctr->active || !sort_step(R.sort_every, ctr->step)) return;
  long long n = ctr->n_total + inject_count(R, ctr->step);
  n = n < R.capacity ? n : R.capacity;
  const PartG<T> A = part_g<T>(R.p[ctr->cur]);
  const PartG<T> B = part_g<T>(R.p[ctr->cur ^ 1]);
  const bool dl = D && (R.physics & PHYS_DELTA);
  __shared__ ScatterLds<T> L;
  const ChunkRange cr = chunk_run(bm, n);
  const int lane = threadIdx.x & 63;
  for (long long ch = cr.beg; ch < cr.end; ch += cr.stride) {
    // the previous chunk has finished reading the staged electrons
    __syncthreads();
    if (threadIdx.x < kNbN) L.cnt[threadIdx.x] = 0;
    const long long i = ch * kBlock + threadIdx.x;
    const uint32_t cell = i < n ? A.cell[i] : kDead;
    const Home hm = make_home(R, __builtin_amdgcn_readfirstlane(G(R.chunk_home)[ch]));
    T v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    uint32_t id = 0;
    int b = -1;
    long long far_slot = -1;
    if (cell != kDead) {
      v[0] = A.ox[i]; v[1] = A.oy[i]; v[2] = A.oz[i];
      v[3] = A.ux[i]; v[4] = A.uy[i]; v[5] = A.uz[i];
      v[6] = A.wn[i]; v[7] = A.tau[i]; id = A.id[i];
      if (dl) v[8] = A.taud[i];
      const int tx = cell_i(cell) >> 2, ty = cell_j(cell) >> 2, tz = cell_k(cell) >> 2;
      b = nb_bin(hm, tx, ty, tz);
      if (b < 0) far_slot = (long long)G(R.tile_start)[tx + R.ntx * (ty + R.nty * tz)] + G(R.far_off)[i];
    }
    __syncthreads();   // counts cleared
    const unsigned rank = wave_rank(L.cnt, b);
    __syncthreads();   // counts complete
    if (threadIdx.x < 64) {
      // exclusive scan of the 125 bin counts: two bins per lane, then the wave
      const int b0 = 2 * lane, b1 = 2 * lane + 1;
      const unsigned c0 = b0 < kNbN ? L.cnt[b0] : 0u, c1 = b1 < kNbN ? L.cnt[b1] : 0u;
      unsigned s = c0 + c1;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const unsigned u = __shfl_up(s, o, 64);
        if (lane >= o) s += u;
      }
      const unsigned ex = s - c0 - c1;
      if (b0 < kNbN) L.start[b0] = ex;
      if (b1 < kNbN) L.start[b1] = ex + c0;
    }
    __syncthreads();   // bin starts ready
    if (b >= 0) {
      const unsigned q = L.start[b] + rank;
#pragma unroll
      for (int f = 0; f < 9; ++f) L.f[f][q] = v[f];
      L.cell[q] = cell;
      L.id[q] = id;
      L.bin[q] = (unsigned char)b;
    } else if (far_slot >= 0 && far_slot < R.capacity) {   // outside the chunk's bins
      B.cell[far_slot] = cell;
      B.ox[far_slot] = v[0]; B.oy[far_slot] = v[1]; B.oz[far_slot] = v[2];
      B.ux[far_slot] = v[3]; B.uy[far_slot] = v[4]; B.uz[far_slot] = v[5];
      B.wn[far_slot] = v[6]; B.tau[far_slot] = v[7]; B.id[far_slot] = id;
      if (dl) B.taud[far_slot] = v[8];
    }
    __syncthreads();   // electrons staged in bin order
    const unsigned nbinned = L.start[kNbN - 1] + L.cnt[kNbN - 1];
    const unsigned q = threadIdx.x;
    if (q < nbinned) {
      const int bq = L.bin[q];
      const int tx = hm.tx + bq % kNb - 2, ty = hm.ty + (bq / kNb) % kNb - 2, tz = hm.tz + bq / (kNb * kNb) - 2;
      const long long slot = (long long)G(R.tile_start)[tx + R.ntx * (ty + R.nty * tz)] +
                             G(R.chunk_base)[ch * kNbN + bq] + (q - L.start[bq]);
      if (slot < R.capacity) {   // counts and scatter agree; the bound is a guard
        B.cell[slot] = L.cell[q];
        B.ox[slot] = L.f[0][q]; B.oy[slot] = L.f[1][q]; B.oz[slot] = L.f[2][q];
        B.ux[slot] = L.f[3][q]; B.uy[slot] = L.f[4][q]; B.uz[slot] = L.f[5][q];
        B.wn[slot] = L.f[6][q]; B.tau[slot] = L.f[7][q]; B.id[slot] = L.id[q];
        if (dl) B.taud[slot] = L.f[8][q];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// delta rays join the run: records grouped by birth tile, ranked by parent
// id inside the tile, appended after the step's survivors
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_spawn_group(const RunDesc* __restrict__ runs,
                                                        const BlockMap* __restrict__ bmap) {
  const BlockMap bm = bmap[blockIdx.x];
  const RunDesc& R = runs[bm.run];
  const auto ctr = G(R.ctr);
  if (!ctr->active || !(R.physics & PHYS_DELTA)) return;
  const long long ns = ctr->n_spawn < R.spawn_cap ? ctr->n_spawn : R.spawn_cap;
  for (long long a = (long long)bm.lb * kBlock + threadIdx.x; a < ns; a += (long long)bm.nb * kBlock) {
    const uint32_t c = G(R.sp_cell)[a];
    const int t = tile_of(R, cell_i(c), cell_j(c), cell_k(c));
    // counting down leaves the tile counts cleared for the next step
    const unsigned k = __hip_atomic_fetch_sub(G(R.sp_cnt) + t, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const long long pos = (long long)G(R.sp_start)[t] + k - 1;
    if (pos >= 0 && pos < ns) {   // counts and records agree; the bound is a guard
      G(R.sp_grp)[pos] = (unsigned)a;
      G(R.sp_gpid)[pos] = G(R.sp_pid)[a];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_spawn_append(const RunDesc* __restrict__ runs,
                                                         const BlockMap* __restrict__ bmap) {
  const BlockMap bm = bmap[blockIdx.x];
  const RunDesc& R = runs[bm.run];
  const auto ctr = G(R.ctr);
  if (!ctr->active || !(R.physics & PHYS_DELTA)) return;
  const long long ns = ctr->n_spawn < R.spawn_cap ? ctr->n_spawn : R.spawn_cap;
  if (ns == 0) return;
  const long long step = ctr->step;
  // the buffer and count the next step starts from (as the end of the step sets them)
  const bool sorted = sort_step(R.sort_every, step);
  long long n0 = ctr->n_total + inject_count(R, step);
  n0 = sorted ? ctr->n_sorted : (n0 < R.capacity ? n0 : R.capacity);
  const PartG<T> P = part_g<T>(R.p[sorted ? ctr->cur ^ 1 : ctr->cur]);
  const long long id0 = ctr->delta_next;
  const long long cap = R.capacity - later_injections(R, step);   // slots of injections to come stay free
  long long acc[L_N + C_N];
#pragma unroll
  for (int i = 0; i < L_N + C_N; ++i) acc[i] = 0;
  const gptr<const unsigned> gpid = G((const unsigned*)R.sp_gpid);
  for (long long g = (long long)bm.lb * kBlock + threadIdx.x; g < ns; g += (long long)bm.nb * kBlock) {
    const unsigned a = G(R.sp_grp)[g];
    if (a >= ns) continue;   // every grouped slot holds a record; the bound is a guard
    const uint32_t c = G(R.sp_cell)[a];
    const int t = tile_of(R, cell_i(c), cell_j(c), cell_k(c));
    const long long st = G(R.sp_start)[t];
    const long long en = t + 1 < R.ntiles ? (long long)G(R.sp_start)[t + 1] : ns;
    const unsigned me = gpid[g];
    long long r = st;
    for (long long j = st; j < en; ++j) r += gpid[j] < me ? 1 : 0;
    const uint32_t id = kDeltaIdBit + (uint32_t)(id0 + r);
    const T ux = G((const T*)R.sp_f[3])[a], uy = G((const T*)R.sp_f[4])[a], uz = G((const T*)R.sp_f[5])[a];
    const T wn = G((const T*)R.sp_f[6])[a];
    const long long slot = n0 + r;
    if (slot < cap) {
      const Uni4<T> u = draws<T>(id, R.seed, step, SLOT_BIRTH);
      P.cell[slot] = c;
      P.ox[slot] = G((const T*)R.sp_f[0])[a];
      P.oy[slot] = G((const T*)R.sp_f[1])[a];
      P.oz[slot] = G((const T*)R.sp_f[2])[a];
      P.ux[slot] = ux; P.uy[slot] = uy; P.uz[slot] = uz;
      P.wn[slot] = wn;
      P.tau[slot] = -m_log((T)1 - u.a);
      P.taud[slot] = -m_log((T)1 - u.b);
      P.id[slot] = id;
    } else {   // no free slot: the delta ray stops in its birth cell
      const T u2 = ux * ux + uy * uy + uz * uz;
      const T e = kinetic(u2, m_sqrt((T)1 + u2)) * wn;
      acc[L_STOPPED] += to_fixed(e * (T)kLedScale);
      acc[L_N + C_DELTA_LOST] += 1;
      atomic_add_i64(&R.heat_acc[cell_i(c) + R.nx * (cell_j(c) + R.ny * cell_k(c))], to_fixed(e * (T)kHeatScale));
      G(R.tdirty)[tile_of(R, cell_i(c), cell_j(c), cell_k(c))] = (int)(step + 1);
    }
  }
  block_flush<L_N, C_N>(acc, R.acc_led, R.events);
}

// ---------------------------------------------------------------------------
// grid kernels
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_zero_step(const RunDesc* __restrict__ runs,
                                                      const BlockMap* __restrict__ bmap) {
  const BlockMap bm = bmap[blockIdx.x];
  const RunDesc& R = runs[bm.run];
  const auto ctr = G(R.ctr);
  if (!ctr->active) return;
  // (the current and heat accumulators are cleared by the gather)
  if (!sort_step(R.sort_every, ctr->step)) return;
  for (int t = bm.lb * kBlock + threadIdx.x; t < R.ntiles; t += bm.nb * kBlock) G(R.tile_cnt)[t] = 0;
}

// The step's current j_h on the Yee edges and collisional heat per cell
// (eq. Ampere_Maxwell, App. A): per tile v of the node grid (node i in tile
// i >> 2, so one more tile per axis than the cells have where n is a
// multiple of 4), each of its nodes sums the accumulator and, of the up to
// eight tiles whose deposit halos hold the node, the partials of those
// claimed this step; each cell its accumulator and its own tile's partial.
// Accumulators are read only where one of those tiles took an atomic this
// step (the others hold zero), and cleared where they were not zero.
constexpr int kGatherU = 4;   // tiles per workgroup iteration of the gather

template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather(const RunDesc* __restrict__ runs,
                                                   const BlockMap* __restrict__ bmap) {
  using A = typename JAcc<T>::type;
  const BlockMap bm = bmap[blockIdx.x];
  const RunDesc& R = runs[bm.run];
  const auto ctr = G(R.ctr);
  if (!ctr->active) return;
  const int stampv = (int)(ctr->step + 1);
  const int nx = R.nx, ny = R.ny, nz = R.nz;
  const int sx = nx + 1, sxy = (nx + 1) * (ny + 1);
  const int gx = (nx >> 2) + 1, gy = (ny >> 2) + 1, gz = (nz >> 2) + 1;
  // component (3: heat; one per wave), node or cell of the tile
  const int c = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), o = threadIdx.x & 63;
  const int ox = o & 3, oy = (o >> 2) & 3, oz = o >> 4;
  // The node's other tile along each axis (-1, +1; 0: none; cells have
  // none) and, for the up to eight tiles u holding it (m: bit 0 x, 1 y, 2 z
  // take the other tile), the node's word in u's partials: pb + p3 u (pb
  // -1: component c's deposit from u never reaches the node).  Every
  // load below is issued unconditionally (lanes with nothing to read load a
  // word they do not use), so that the loads of an iteration are all in
  // flight together instead of each waiting at the end of its branch.
  const bool hc = c == 3;
  const int ax = hc ? 0 : (ox == 0 ? -1 : (ox == kTile - 1 ? 1 : 0));
  const int ay = hc ? 0 : (oy == 0 ? -1 : (oy == kTile - 1 ? 1 : 0));
  const int az = hc ? 0 : (oz == 0 ? -1 : (oz == kTile - 1 ? 1 : 0));
  int pb[8];
#pragma unroll
  for (int m = 0; m < 8; ++m)
    pb[m] = hc ? o : pj_word(-(m & 1 ? ax : 0), -(m & 2 ? ay : 0), -(m & 4 ? az : 0), hc ? 0 : c, ox, oy, oz);
  const long long pstr = hc ? kTile * kTile * kTile : 3 * kPjWords;   // words per tile
  const gptr<const A> pj = G((const A*)R.pj);
  const gptr<const long long> ph = G((const long long*)R.ph);
  // A workgroup sweeps segments of rows of tiles along x (up to 8 groups of
  // kGatherU tiles, one group per iteration), so that the partials and the
  // node rows are read as sequential streams; the workgroups stride over
  // the segments, so that those running at a time share one window of the
  // grid.  The claims and atomic marks of the 27 tiles around each tile of
  // an iteration are staged in LDS one iteration ahead (claim: low bit set
  // if claimed this step; mark: bit 1).  A node's accumulator is read only
  // if one of its tiles is marked; else it loads a word it does not use.
  const uint32_t ngr = (uint32_t)(gx + kGatherU - 1) / kGatherU, nrows = (uint32_t)gy * gz;
  const uint32_t nseg = gather_segments(R.nx), kseg = (ngr + nseg - 1) / nseg;   // segments per row, groups per segment
  const uint32_t nunit = nrows * nseg;
  const uint32_t myunits = (uint32_t)bm.lb < nunit ? (nunit - 1 - bm.lb) / bm.nb + 1 : 0;
  const uint32_t nit = myunits * kseg;
  auto place = [&](uint32_t it, int& vx0, int& vy, int& vz) {   // first tile of iteration it's group
    const uint32_t unit = bm.lb + (it / kseg) * bm.nb;
    const uint32_t row = unit / nseg;
    const uint32_t vzu = R.fd_gy.div(row);
    vy = (int)(row - vzu * (uint32_t)gy);
    vz = (int)vzu;
    vx0 = (int)((unit - row * nseg) * kseg + it % kseg) * kGatherU;
  };
  __shared__ int st[2][kGatherU][27];
  const bool stager = threadIdx.x < 27 * kGatherU;
  auto claim_of = [&](uint32_t it) -> int {   // the flags a stager thread stages for iteration it
    if (it >= nit) return 0;
    const int g = (int)threadIdx.x / 27, n = (int)threadIdx.x % 27;
    int vx0, vy, vz;
    place(it, vx0, vy, vz);
    const int ux = vx0 + g + n % 3 - 1, uy = vy + (n / 3) % 3 - 1, uz = vz + n / 9 - 1;
    const bool in = ux >= 0 && uy >= 0 && uz >= 0 && ux < R.ntx && uy < R.nty && uz < R.ntz;
    const long long u = in ? ux + (long long)R.ntx * (uy + (long long)R.nty * uz) : 0;
    const int cl = G((const int*)R.tstamp)[u], mk = G((const int*)R.tdirty)[u];
    return in ? (cl == stampv ? 1 : 0) | (mk == stampv ? 2 : 0) : 0;
  };
  if (stager) st[0][threadIdx.x / 27][threadIdx.x % 27] = claim_of(0);
  __syncthreads();
  // the waves of the current and of the heat take separate loops (the
  // component is uniform per wave), each with the same barriers
  auto sweep = [&](auto hc_tag) {
    constexpr bool HC = decltype(hc_tag)::value;
    const gptr<long long> acc = G(HC ? R.heat_acc : R.Jacc[HC ? 0 : c]);
    const gptr<long long> out = G(HC ? R.ion_heat : R.J[HC ? 0 : c]);
    int buf = 0;
    for (uint32_t it = 0; it < nit; ++it, buf ^= 1) {
      const int nxt = stager ? claim_of(it + 1) : 0;   // lands while this iteration's loads run
      int vx0, vy, vz;
      place(it, vx0, vy, vz);
      bool in[kGatherU], rd[kGatherU];
      int at[kGatherU], usem[kGatherU];
      long long a0[kGatherU];
      using W = std::conditional_t<HC, long long, A>;   // partials: 32-bit words in FP32 runs
      W w[kGatherU][HC ? 1 : 8];
#pragma unroll
      for (int g = 0; g < kGatherU; ++g) {
        const int vx = vx0 + g;
        const int i = kTile * vx + ox, j = kTile * vy + oy, k = kTile * vz + oz;
        in[g] = HC ? (i < nx && j < ny && k < nz) : (i <= nx && j <= ny && k <= nz);
        at[g] = in[g] ? (HC ? i + nx * (j + ny * k) : i + sx * j + sxy * k) : 0;
        usem[g] = 0;
        rd[g] = false;
#pragma unroll
        for (int m = 0; m < (HC ? 1 : 8); ++m) {
          const int dx = m & 1 ? ax : 0, dy = m & 2 ? ay : 0, dz = m & 4 ? az : 0;
          const bool holds = in[g] && (!(m & 1) || ax) && (!(m & 2) || ay) && (!(m & 4) || az);
          const bool part = pb[m] >= 0;   // the holder's partials of component c reach the node
          const int fl = st[buf][g][13 + dx + 3 * dy + 9 * dz];
          const bool use = holds && part && (fl & 1);
          rd[g] |= holds && (fl & 2);
          const long long u = (vx + dx) + (long long)R.ntx * ((vy + dy) + (long long)R.nty * (vz + dz));
          const long long wa = use ? pb[m] + u * pstr : 0;
          if constexpr (HC) w[g][m] = ph[wa];
          else w[g][m] = pj[wa];
          usem[g] |= use ? 1 << m : 0;
        }
        a0[g] = acc[rd[g] ? at[g] : 0];
      }
      __builtin_amdgcn_sched_barrier(0);   // every load above is issued before the first sum waits
#pragma unroll
      for (int g = 0; g < kGatherU; ++g) {
        long long a = 0;
#pragma unroll
        for (int m = 0; m < (HC ? 1 : 8); ++m) a += (usem[g] >> m) & 1 ? w[g][m] : 0LL;
        if (!HC) a *= (1LL << JAcc<T>::shift);
        const long long a0g = rd[g] ? a0[g] : 0LL;
        if (in[g]) {
          if (a0g != 0) acc[at[g]] = 0;
          out[at[g]] = a0g + a;
        }
      }
      if (stager) st[buf ^ 1][threadIdx.x / 27][threadIdx.x % 27] = nxt;
      __syncthreads();
    }
  };
  if (hc) sweep(std::true_type{});
  else sweep(std::false_type{});
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// E = eta_edge (curl B / mu0 - j_h) on the three edge families
template <typename T>
__global__ __launch_bounds__(kBlock) void k_ohm(const RunDesc* __restrict__ runs,
                                                const BlockMap* __restrict__ bmap, int sub) {
  const BlockMap bm = bmap[blockIdx.x];
  const RunDesc& R = runs[bm.run];
  if (!G(R.ctr)->active || sub >= R.n_sub || !(R.physics & PHYS_EVOLVE_E)) return;
  const int nx = R.nx, ny = R.ny, nz = R.nz;
  const int sx = nx + 1, sxy = (nx + 1) * (ny + 1);
  const gptr<const T> Bx = G((const T*)R.B[0]), By = G((const T*)R.B[1]), Bz = G((const T*)R.B[2]);
  const gptr<T> Ex = G((T*)R.E[0]), Ey = G((T*)R.E[1]), Ez = G((T*)R.E[2]);
  const gptr<const long long> Jx = G((const long long*)R.J[0]), Jy = G((const long long*)R.J[1]),
                              Jz = G((const long long*)R.J[2]);
  const gptr<const double> eta = G((const double*)R.eta[G(R.ctr)->step & 1]);
  const double inv_dx = 1.0 / R.dx, inv_mu0 = 1.0 / kMu0, ju = R.j_unit;
  const uint32_t nn = (uint32_t)R.nodes;   // < 2^31 (checked at init)
  auto ce = [&](int i, int j, int k) { return eta[i + nx * (j + ny * k)]; };
  for (uint32_t t = bm.lb * kBlock + threadIdx.x; t < nn; t += bm.nb * kBlock) {
    const uint32_t q = R.fd_sx.div(t), kk = R.fd_sy.div(q);
    const int i = (int)(t - q * (uint32_t)sx);
    const int j = (int)(q - kk * (uint32_t)(ny + 1));
    const int k = (int)kk;
    const int idx = (int)t;
    const int jm = clampi(j - 1, 0, ny - 1), jc = clampi(j, 0, ny - 1);
    const int km = clampi(k - 1, 0, nz - 1), kc = clampi(k, 0, nz - 1);
    const int im = clampi(i - 1, 0, nx - 1), ic = clampi(i, 0, nx - 1);
    if (i < nx) {   // Ex at (i+1/2, j, k): dBz/dy - dBy/dz
      const T bzp = j < ny ? Bz[idx] : -Bz[idx - sx];
      const T bzm = j > 0 ? Bz[idx - sx] : -Bz[idx];
      const T byp = k < nz ? By[idx] : -By[idx - sxy];
      const T bym = k > 0 ? By[idx - sxy] : -By[idx];
      const double curl = (double)((bzp - bzm) - (byp - bym)) * inv_dx;
      const double ee = 0.25 * (ce(i, jm, km) + ce(i, jc, km) + ce(i, jm, kc) + ce(i, jc, kc));
      Ex[idx] = (T)(ee * (curl * inv_mu0 - (double)Jx[idx] * ju));
    }
    if (j < ny) {   // Ey at (i, j+1/2, k): dBx/dz - dBz/dx
      const T bxp = k < nz ? Bx[idx] : -Bx[idx - sxy];
      const T bxm = k > 0 ? Bx[idx - sxy] : -Bx[idx];
      const T bzp = i < nx ? Bz[idx] : -Bz[idx - 1];
      const T bzm = i > 0 ? Bz[idx - 1] : -Bz[idx];
      const double curl = (double)((bxp - bxm) - (bzp - bzm)) * inv_dx;
      const double ee = 0.25 * (ce(im, j, km) + ce(ic, j, km) + ce(im, j, kc) + ce(ic, j, kc));
      Ey[idx] = (T)(ee * (curl * inv_mu0 - (double)Jy[idx] * ju));
    }
    if (k < nz) {   // Ez at (i, j, k+1/2): dBy/dx - dBx/dy
      const T byp = i < nx ? By[idx] : -By[idx - 1];
      const T bym = i > 0 ? By[idx - 1] : -By[idx];
      const T bxp = j < ny ? Bx[idx] : -Bx[idx - sx];
      const T bxm = j > 0 ? Bx[idx - sx] : -Bx[idx];
      const double curl = (double)((byp - bym) - (bxp - bxm)) * inv_dx;
      const double ee = 0.25 * (ce(im, jm, k) + ce(ic, jm, k) + ce(im, jc, k) + ce(ic, jc, k));
      Ez[idx] = (T)(ee * (curl * inv_mu0 - (double)Jz[idx] * ju));
    }
  }
}

// B -= (dt / n_sub) curl E on the three face families
template <typename T>
__global__ __launch_bounds__(kBlock) void k_faraday(const RunDesc* __restrict__ runs,
                                                    const BlockMap* __restrict__ bmap, int sub) {
  const BlockMap bm = bmap[blockIdx.x];
  const RunDesc& R = runs[bm.run];
  if (!G(R.ctr)->active || sub >= R.n_sub || !(R.physics & PHYS_EVOLVE_B)) return;
  const int nx = R.nx, ny = R.ny, nz = R.nz;
  const int sx = nx + 1, sxy = (nx + 1) * (ny + 1);
  const gptr<const T> Ex = G((const T*)R.E[0]), Ey = G((const T*)R.E[1]), Ez = G((const T*)R.E[2]);
  const gptr<T> Bx = G((T*)R.B[0]), By = G((T*)R.B[1]), Bz = G((T*)R.B[2]);
  const T h = (T)(R.dt / R.n_sub / R.dx);
  const uint32_t nn = (uint32_t)R.nodes;   // < 2^31 (checked at init)
  for (uint32_t t = bm.lb * kBlock + threadIdx.x; t < nn; t += bm.nb * kBlock) {
    const uint32_t q = R.fd_sx.div(t), kk = R.fd_sy.div(q);
    const int i = (int)(t - q * (uint32_t)sx);
    const int j = (int)(q - kk * (uint32_t)(ny + 1));
    const int k = (int)kk;
    const int idx = (int)t;
    if (j < ny && k < nz)   // Bx: dEz/dy - dEy/dz
      Bx[idx] -= h * ((Ez[idx + sx] - Ez[idx]) - (Ey[idx + sxy] - Ey[idx]));
    if (i < nx && k < nz)   // By: dEx/dz - dEz/dx
      By[idx] -= h * ((Ex[idx + sxy] - Ex[idx]) - (Ez[idx + 1] - Ez[idx]));
    if (i < nx && j < ny)   // Bz: dEy/dx - dEx/dy
      Bz[idx] -= h * ((Ey[idx + 1] - Ey[idx]) - (Ex[idx + sx] - Ex[idx]));
  }
}

// Ohmic + collisional heating, exchange and resistivity of the solid cells
// (FP64).  MIX: some run of the launch has a compound solid (the
// single-element instance keeps the compound code out of its registers).
template <bool MIX>
__global__ __launch_bounds__(kBlock) void k_heat(const RunDesc* __restrict__ runs,
                                                 const BlockMap* __restrict__ bmap) {
  const BlockMap bm = bmap[blockIdx.x];
  const RunDesc& R = runs[bm.run];
  if (!G(R.ctr)->active || !(R.physics & PHYS_HEAT)) return;
  const int nx = R.nx, ny = R.ny;
  const int sx = nx + 1, sxy = (nx + 1) * (ny + 1);
  const int w = R.ix_hi - R.ix_lo;
  const uint32_t ns = (uint32_t)w * ny * R.nz;   // < 2^31 (checked at init)
  const double ju = 0.25 * R.j_unit, dV = R.dx * R.dx * R.dx;
  const bool fixed = R.eta_fixed > 0.0;
  const bool want_fs = (R.physics & PHYS_FSIGMA) != 0;
  // this step's resistivity in, the next step's out: the field sub-cycles,
  // which read this step's, may run at the same time
  const long long step = G(R.ctr)->step;
  const gptr<const double> eta_in = G((const double*)R.eta[step & 1]);
  const gptr<double> eta_out = G(R.eta[(step + 1) & 1]);
  const Solid& sol = R.solid;   // read in place: a copy of the constants would take registers
  for (uint32_t t = bm.lb * kBlock + threadIdx.x; t < ns; t += bm.nb * kBlock) {
    const uint32_t q = R.fd_w.div(t), kk = R.fd_ny.div(q);
    const int i = R.ix_lo + (int)(t - q * (uint32_t)w);
    const int j = (int)(q - kk * (uint32_t)ny);
    const int k = (int)kk;
    const int c = i + nx * (j + ny * k);
    const int n = i + sx * j + sxy * k;
    const gptr<const long long> Jx = G((const long long*)R.J[0]), Jy = G((const long long*)R.J[1]),
                                Jz = G((const long long*)R.J[2]);
    const double jx = (double)(Jx[n] + Jx[n + sx] + Jx[n + sxy] + Jx[n + sx + sxy]) * ju;
    const double jy = (double)(Jy[n] + Jy[n + 1] + Jy[n + sxy] + Jy[n + 1 + sxy]) * ju;
    const double jz = (double)(Jz[n] + Jz[n + 1] + Jz[n + sx] + Jz[n + 1 + sx]) * ju;
    double Te = G(R.Te)[c], Ti = G(R.Ti)[c], eta = eta_in[c], fs = 1.0;
    const double j2 = jx * jx + jy * jy + jz * jz, qh = (double)G(R.ion_heat)[c] * R.heat_unit;
    if (!MIX || R.mix.n == 1) heat_cell(sol, Te, Ti, eta, j2, qh, R.dt, dV, fixed, want_fs, fs);
    else heat_cell_mix(R.mix, Te, Ti, eta, j2, qh, R.dt, dV, fixed, false, fs);
    if (want_fs) {
      if (R.precision == 0) G((double*)R.fsig)[c] = fs;
      else G((float*)R.fsig)[c] = (float)fs;
    }
    G(R.Te)[c] = Te;
    G(R.Ti)[c] = Ti;
    eta_out[c] = eta;
  }
}

__device__ __forceinline__ void kahan(gptr<double> s, gptr<double> c, double v) {
  const double y = v - *c;
  const double t = *s + y;
  *c = (t - *s) - y;
  *s = t;
}

// Per-step integer accumulators -> FP64 Kahan totals (fixed order), reset.
__global__ __launch_bounds__(kBlock) void k_finalize(const RunDesc* __restrict__ runs,
                                                     const BlockMap* __restrict__ bmap) {
  const BlockMap bm = bmap[blockIdx.x];
  const RunDesc& R = runs[bm.run];
  const auto ctr = G(R.ctr);
  if (!ctr->active) return;
  const int nbin = R.nE * R.nth;
  const long long nh = 2LL * nbin + 4;
  for (long long b = (long long)bm.lb * kBlock + threadIdx.x; b < nh; b += (long long)bm.nb * kBlock) {
    long long x = 0;
    for (int c = 0; c < kHistCopies; ++c) {
      const gptr<long long> a = G(R.acc_hist) + c * R.hist_stride + b;
      const long long v = *a;
      if (v != 0) {
        x += v;
        *a = 0;
      }
    }
    if (x == 0) continue;
    bool is_energy;
    if (b < nbin) is_energy = true;
    else if (b < 2 * nbin) is_energy = false;
    else is_energy = ((b - 2 * nbin) & 1) == 0;
    kahan(G(R.tot_hist) + b, G(R.tot_hist_c) + b, (double)x * (is_energy ? R.led_unit : R.cnt_unit));
  }
  if (bm.lb == 0 && threadIdx.x < L_N) {
    const int l = threadIdx.x;
    const long long x = G(R.acc_led)[l];
    const double v = (double)x * R.led_unit;
    if (x != 0) kahan(G(R.tot_led) + l, G(R.tot_led_c) + l, v);
    G(R.acc_led)[l] = 0;
    if (l == L_PHOTON_THR) {
      const long long step = ctr->step;
      if (step < R.series_len) G(R.series)[step] = v;
    }
  }
}

// End of step: particle count, step counter, engine bookkeeping (one
// single-thread block per run).
__global__ void k_advance(const RunDesc* __restrict__ runs, const BlockMap* __restrict__ bmap) {
  const BlockMap bm = bmap[blockIdx.x];
  if (threadIdx.x != 0) return;
  const RunDesc& R = runs[bm.run];
  const gptr<Counters> c = G(R.ctr);
  if (!c->active) return;
  if (sort_step(R.sort_every, c->step)) {
    c->n_total = c->n_sorted;   // the scatter kept the alive electrons only
    c->cur ^= 1;
  } else {
    const long long n = c->n_total + inject_count(R, c->step);
    c->n_total = n < R.capacity ? n : R.capacity;
  }
  if (R.physics & PHYS_DELTA) {   // the step's delta rays were appended
    const long long ns = c->n_spawn < R.spawn_cap ? c->n_spawn : R.spawn_cap;
    const long long n = c->n_total + ns, cap = R.capacity - later_injections(R, c->step);
    c->n_total = n < cap ? n : (c->n_total > cap ? c->n_total : cap);
    c->delta_next += ns;
    c->n_spawn = 0;
  }
  c->step += 1;
  if (c->steps_left > 0) {
    c->steps_left -= 1;
    if (c->steps_left == 0) c->active = 0;
  }
}

// Kinetic energy and alive count: per-block partial sums (fixed tree order).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_kinetic(const RunDesc* __restrict__ runs, int run) {
  const RunDesc& R = runs[run];
  const auto ctr = G(R.ctr);
  const long long n = ctr->n_total;
  const PartG<T> P = part_g<T>(R.p[ctr->cur]);
  double s = 0.0, cnt = 0.0;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) {
    if (P.cell[i] == kDead) continue;
    const T ux = P.ux[i], uy = P.uy[i], uz = P.uz[i];
    const double u2 = (double)ux * ux + (double)uy * uy + (double)uz * uz;
    s += (double)P.wn[i] * (u2 / (1.0 + sqrt(1.0 + u2)));
    cnt += 1.0;
  }
  __shared__ double sm[2][kBlock];
  sm[0][threadIdx.x] = s;
  sm[1][threadIdx.x] = cnt;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      sm[0][threadIdx.x] += sm[0][threadIdx.x + o];
      sm[1][threadIdx.x] += sm[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    G(R.red)[2 * blockIdx.x] = sm[0][0];
    G(R.red)[2 * blockIdx.x + 1] = sm[1][0];
  }
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
template <typename T>
static void launch_step_t(const LaunchSet& L, hipStream_t s, int max_sub) {
  hipLaunchKernelGGL(k_zero_step, dim3(L.zero.nb), dim3(kBlock), 0, s, L.runs, L.zero.map);
  hipLaunchKernelGGL(k_inject<T>, dim3(L.inject.nb), dim3(kBlock), 0, s, L.runs, L.inject.map);
  if (L.ev_start) (void)hipEventRecord(L.ev_start, s);
  switch ((L.delta ? kVarDelta : 0) | (L.urban ? kVarUrban : 0)) {
    case 0: hipLaunchKernelGGL((k_particle<T, 0>), dim3(L.particle.nb), dim3(kBlock), 0, s, L.runs, L.particle.map); break;
    case kVarDelta:
      hipLaunchKernelGGL((k_particle<T, kVarDelta>), dim3(L.particle.nb), dim3(kBlock), 0, s, L.runs, L.particle.map);
      break;
    case kVarUrban:
      hipLaunchKernelGGL((k_particle<T, kVarUrban>), dim3(L.particle.nb), dim3(kBlock), 0, s, L.runs, L.particle.map);
      break;
    default:
      hipLaunchKernelGGL((k_particle<T, kVarDelta | kVarUrban>), dim3(L.particle.nb), dim3(kBlock), 0, s, L.runs,
                         L.particle.map);
  }
  if (L.ev_stop) (void)hipEventRecord(L.ev_stop, s);
  auto gather = [&]() { hipLaunchKernelGGL(k_gather<T>, dim3(L.gather.nb), dim3(kBlock), 0, s, L.runs, L.gather.map); };
  // The gather of the step's current and heat comes first (delta-ray
  // appends can book a lost delta ray's energy as heat: runs with delta rays
  // gather after them).  Then the sort (scans, scatter), the field
  // sub-cycles and the heating read and write disjoint data (the heating
  // writes the next step's resistivity), so with two more streams the grid
  // kernels run beside the HBM-bound scatter; runs with delta rays keep one
  // stream.  (Running the gather beside the scatter instead measured slower:
  // the kernels after it then overlap less.)
  if (!L.delta) gather();
  const bool split = L.side && L.side2 && L.ev_fork && L.ev_join && L.ev_join2 && !L.delta;
  auto fields = [&](hipStream_t g) {
    for (int k = 0; k < max_sub; ++k) {
      hipLaunchKernelGGL(k_ohm<T>, dim3(L.grid.nb), dim3(kBlock), 0, g, L.runs, L.grid.map, k);
      hipLaunchKernelGGL(k_faraday<T>, dim3(L.grid.nb), dim3(kBlock), 0, g, L.runs, L.grid.map, k);
    }
  };
  auto heating = [&](hipStream_t g) {
    if (L.compound) hipLaunchKernelGGL(k_heat<true>, dim3(L.cells.nb), dim3(kBlock), 0, g, L.runs, L.cells.map);
    else hipLaunchKernelGGL(k_heat<false>, dim3(L.cells.nb), dim3(kBlock), 0, g, L.runs, L.cells.map);
  };
  if (L.sort) {
    hipLaunchKernelGGL(k_scan_reduce, dim3(L.scan.nb), dim3(kBlock), 0, s, L.runs, L.scan.map, 0);
    hipLaunchKernelGGL(k_scan_blocks, dim3(L.scan1.nb), dim3(kBlock), 0, s, L.runs, L.scan1.map, 0);
    hipLaunchKernelGGL(k_scan_tiles, dim3(L.scan.nb), dim3(kBlock), 0, s, L.runs, L.scan.map, 0);
  }
  // the fork comes after the short scans: launched beside the grid kernels,
  // whose workgroups fill the machine, they would wait for free slots
  if (split) {   // field sub-cycles and heating each on a stream of their own
    (void)hipEventRecord(L.ev_fork, s);
    (void)hipStreamWaitEvent(L.side, L.ev_fork, 0);
    (void)hipStreamWaitEvent(L.side2, L.ev_fork, 0);
    heating(L.side2);
    fields(L.side);
  }
  if (L.sort) {
    if (L.delta) hipLaunchKernelGGL((k_scatter<T, true>), dim3(L.particle.nb), dim3(kBlock), 0, s, L.runs, L.particle.map);
    else hipLaunchKernelGGL((k_scatter<T, false>), dim3(L.particle.nb), dim3(kBlock), 0, s, L.runs, L.particle.map);
  }
  if (L.delta) {
    hipLaunchKernelGGL(k_scan_reduce, dim3(L.scan.nb), dim3(kBlock), 0, s, L.runs, L.scan.map, 1);
    hipLaunchKernelGGL(k_scan_blocks, dim3(L.scan1.nb), dim3(kBlock), 0, s, L.runs, L.scan1.map, 1);
    hipLaunchKernelGGL(k_scan_tiles, dim3(L.scan.nb), dim3(kBlock), 0, s, L.runs, L.scan.map, 1);
    hipLaunchKernelGGL(k_spawn_group, dim3(L.inject.nb), dim3(kBlock), 0, s, L.runs, L.inject.map);
    hipLaunchKernelGGL(k_spawn_append<T>, dim3(L.inject.nb), dim3(kBlock), 0, s, L.runs, L.inject.map);
    gather();
  }
  if (split) {
    (void)hipEventRecord(L.ev_join, L.side);
    (void)hipEventRecord(L.ev_join2, L.side2);
    (void)hipStreamWaitEvent(s, L.ev_join, 0);
    (void)hipStreamWaitEvent(s, L.ev_join2, 0);
  } else {
    fields(s);
    heating(s);
  }
  hipLaunchKernelGGL(k_finalize, dim3(L.fin.nb), dim3(kBlock), 0, s, L.runs, L.fin.map);
  hipLaunchKernelGGL(k_advance, dim3(L.adv.nb), dim3(64), 0, s, L.runs, L.adv.map);
}

void launch_step(const LaunchSet& L, hipStream_t s, int precision, int max_sub) {
  if (precision == 0) launch_step_t<double>(L, s, max_sub);
  else launch_step_t<float>(L, s, max_sub);
}

void launch_kinetic(const RunDesc* runs, int run, int nblocks, hipStream_t s, int precision) {
  if (precision == 0) hipLaunchKernelGGL(k_kinetic<double>, dim3(nblocks), dim3(kBlock), 0, s, runs, run);
  else hipLaunchKernelGGL(k_kinetic<float>, dim3(nblocks), dim3(kBlock), 0, s, runs, run);
}

}  // namespace hyb
