// Kernels of one RK3 substep (Sec. 2.4, Eq. (16), with the projection of Sec. 2.1):
//   momentum   explicit right-hand side, RK combination, implicit immersed-boundary update
//   cfr        flow-rate reduction -> mean pressure gradient
//   div_fftx   divergence of u* fused with the real FFT along x
//   fftz       complex FFT along z (forward / inverse)
//   tri        wall-normal tridiagonal solve per Fourier mode (FP64 arithmetic)
//   ifftx      inverse real FFT along x -> phi
//   correct    velocity correction, reset of external faces, pressure update
#include "fft_lds.h"
#include "ibm_internal.h"

namespace {

constexpr int BX = 64;  // x points per block row (one wavefront)
constexpr int BZ = 4;   // z rows per block

__device__ __forceinline__ int wrap_p(int i, int n) { return (i + 1 == n) ? 0 : i + 1; }
__device__ __forceinline__ int wrap_m(int i, int n) { return (i == 0) ? n - 1 : i - 1; }

// Instance of block b in a batched launch (boff[i] <= b < boff[i+1], boff[0] = 0): read
// from the table of every block's instance that follows the ninst + 1 offsets (one load,
// where a binary search over the offsets made a chain of dependent loads at every block's
// start).
__device__ __forceinline__ int batch_instance(const int* __restrict__ boff, int ninst, int b) {
  return boff[ninst + 1 + b];
}

// ---------------------------------------------------------------------------------------
// momentum: H = -N(u) + nu L(u) at internal points (external/ghost neighbours are zero),
// r = dt (a_k H + b_k H_prev) - c_k dt G p, and the predictor u* = (B u + r) / A of
// Eq. (16) (B = A = 1 away from the wall: u* = u + r).  Per-block partial sums of u*
// over internal u points feed the flow-rate reduction.
//
// The projection of the previous substep is folded in: the state it would have written,
//   u = u*' - Pi' c' dt (non-IBM internal u) - c' dt G phi  on internal faces, 0 elsewhere,
//   p = p' + phi  on internal cells, 0 elsewhere,
// is formed here from the previous predictor u*', the increment phi and the previous
// pressure p' as the planes are loaded (c' = c_{k-1}, Pi' = Pi_{k-1}); p is also written
// out (f.pn) for the next substep.
//
// A block owns an MX x MZ (x, z) column of cells (64 x 4 by default; a wavefront is one
// 64-wide row chunk) and marches through a chunk of y planes.  u, v, w, p live in a ring of four LDS planes (j-1, j, j+1 and the one being
// filled) with a halo of one row in z and two columns in x (so that the tile is made of
// whole, aligned pairs of x-adjacent values: every thread loads one pair of each field
// with one vector load).  The loads of plane j+2 are issued before the arithmetic of
// plane j and their corrected values written to the ring slot of plane j-2 afterwards.
// Planes outside the box (ghost rows, the north wall face of v) are zero.
// ---------------------------------------------------------------------------------------
constexpr int MX = 64, MZ = 4;   // default tile (and the batched launches' tile)
template <int TX, int TZ>
struct MomTile {
  static constexpr int HX = TX + 4, HZ = TZ + 2, TILE = HX * HZ;   // 408 values at 64 x 4
  static constexpr int PAIRS = TILE / 2;                           // 204 pairs, one per thread
  static constexpr int THREADS = TX * TZ;
  static_assert(PAIRS <= THREADS, "one tile pair per thread");
  static_assert(TX % 64 == 0, "whole 64-wide row chunks per block row");
};

template <typename T>
struct alignas(2 * sizeof(T)) Pair {
  T x, y;
};
template <typename T>
__device__ __forceinline__ Pair<T> ld_pair(const T* p) { return *reinterpret_cast<const Pair<T>*>(p); }

// Loaded inputs of one pair of x-adjacent tile values (x, x+1): previous predictor,
// previous pressure, phi, phi at x-2 and x-1 (the west neighbours), phi of the back row
// and of the plane below, the two tags (x in the low byte).
template <typename T>
struct TileRaw {
  Pair<T> us, vs, ws, pp, ph, phw, phz, phy;
  uint16_t tg, keep;   // loaded tags; mask applied to them when the pair is stored
};

// The 1-D grid's blocks are dealt round-robin to the 8 XCDs (block b to XCD b mod 8, each
// with its own L2).  Tiles are numbered x fastest, then z, then y chunk.  With xcd_order
// block b takes tile (b mod 8) * (share of one XCD) + b / 8, so that each XCD works
// through a contiguous run of tiles and neighbouring tiles, which load each other's
// halos, share an L2; without it block b takes tile b (the XCDs interleave, which keeps
// concurrent HBM accesses close together).
constexpr int NXCD = 8;

template <typename T, bool SY, int MXT = MX, int MZT = MZ, int PF = 1>
__device__ __forceinline__ void k_momentum_body(GridParams g, Fields<T> f, IbmLists L, StageConsts s, int jc,
                                                 int ntx, int ntz, int xcd_order, const double* __restrict__ pi_prev,
                                                 double ckdt_prev, double* __restrict__ qpart, int bid_x, int bid_y, int nblk) {
  using TL = MomTile<MXT, MZT>;
  constexpr int MHX = TL::HX, MTILE = TL::TILE, MPAIRS = TL::PAIRS;
  __shared__ __align__(16) T ring[4][4][MTILE];   // [field u,v,w,p][slot][tile]
  __shared__ double red[TL::THREADS / 64];
  const int tx = threadIdx.x, tz = threadIdx.y, tid = tz * MXT + tx;
  const int lane = tx & 63;
  const int nx = g.nx, nz = g.nz, ny1 = g.ny1, plane = nx * nz;
  int bx, bz, by;
  {
    const int nb = nblk, b = bid_x;
    const int lsx = (xcd_order >> MOM_SUPER_SHIFT) & 3, lsz = (xcd_order >> (MOM_SUPER_SHIFT + 2)) & 3;
    if (lsx | lsz) {
      // super-tiles of 2^lsx x 2^lsz tiles, dealt round-robin to the XCDs; the members of
      // one super-tile are consecutive blocks of one XCD (dispatched together, so that
      // they share their common halo rows and columns through that XCD's L2)
      const int sx = 1 << lsx, ms = 1 << (lsx + lsz);
      const int xcd = b % NXCD, sq = b / NXCD;
      const int r = sq >> (lsx + lsz), m = sq & (ms - 1);
      const int qs = r * NXCD + xcd;
      const int nsx = ntx >> lsx, nsz = ntz >> lsz;
      bx = (qs % nsx) * sx + (m & (sx - 1));
      bz = ((qs / nsx) % nsz) * (1 << lsz) + (m >> lsx);
      by = qs / (nsx * nsz);
    } else {
      const int xcd = b % NXCD, q = nb / NXCD, rem = nb % NXCD;
      const int t = (xcd_order & MOM_XCD_CONTIG) ? xcd * q + min(xcd, rem) + b / NXCD : b;
      bx = t % ntx;
      bz = (t / ntx) % ntz;
      by = t / (ntx * ntz);
    }
  }
  const int i0 = bx * MXT, k0 = bz * MZT;
  const int chk = (i0 + tx) >> 6;   // this wavefront's 64-wide chunk of the row
  const int j0 = by * jc;
  const int j1 = min(j0 + jc, ny1);
  const int i = i0 + tx, k = k0 + tz;
  const bool act = (i < nx) && (k < nz);
  // this thread's tile pair -> offsets inside a plane (periodic wrap in x and z) of itself,
  // of the pair west of it and of the pair in the back row; threads past the tile repeat
  // the last pair's loads (cache hits) and write nothing
  const bool has = tid < MPAIRS;
  int off, offw, offb;
  {
    const int pidx = has ? tid : MPAIRS - 1;
    const int lz = pidx / (MHX / 2), lx = 2 * (pidx - lz * (MHX / 2));
    int gz = (k0 - 1 + lz) % nz;
    if (gz < 0) gz += nz;
    int gx = (i0 - 2 + lx) % nx;   // even: nx is even
    if (gx < 0) gx += nx;
    off = gz * nx + gx;
    offw = gz * nx + (gx == 0 ? nx - 2 : gx - 2);
    offb = (gz == 0 ? nz - 1 : gz - 1) * nx + gx;
  }
  const T pick = T(pi_prev[0] * ckdt_prev), ckp = T(ckdt_prev);
  // immersed walls' velocity (held by the external points inside the box)
  const T ubw = T(L.wallv[0]), vbw = T(L.wallv[1]), wbw = T(L.wallv[2]);
  const T idx = T(g.idx), idy = T(g.idy), idz = T(g.idz);
  // phi of the plane below this thread's pair (the v correction's south neighbour) is
  // kept from the previous plane instead of being loaded again; only the first plane of
  // the prologue loads it (with_phy).
  Pair<T> phprev = {T(0), T(0)};
  // The loads are unconditional (a plane outside the box reads the nearest one and a zero
  // tag then zeroes the values): without branches around them the compiler can count
  // them, so that waiting for loads issued earlier does not wait for these.
  auto fetch = [&](int jj, TileRaw<T>& q, bool with_phy) {
    const bool inb = jj >= 0 && jj < ny1;
    const int b = (jj < 0 ? 0 : (jj < ny1 ? jj : ny1 - 1)) * plane;
    q.us = ld_pair(f.usp + b + off);
    q.vs = ld_pair(f.vsp + b + off);
    q.ws = ld_pair(f.wsp + b + off);
    q.pp = ld_pair(f.pp + b + off);
    q.ph = ld_pair(f.phi + b + off);
    q.phw = ld_pair(f.phi + b + offw);
    q.phz = ld_pair(f.phi + b + offb);
    q.phy = Pair<T>{T(0), T(0)};
    if (with_phy && inb && jj > 0) q.phy = ld_pair(f.phi + b - plane + off);
    const uint16_t t = *reinterpret_cast<const uint16_t*>(f.tag + b + off);
    // above a free-slip north face the row mirrors the top row's u and w (the clamped
    // load is that row); v on the face and p are zero there
    const uint16_t keep = (g.top_fs && jj == ny1) ? uint16_t(~((TAG_V | TAG_VI | TAG_P) * 0x0101u)) : uint16_t(0);
    // (with loads two planes ahead the mask is applied where the pair is stored: an
    // operation on the loaded tag here would wait for this plane's loads at once)
    if constexpr (PF == 2) {
      q.tg = t;
      q.keep = inb ? uint16_t(0xffff) : keep;
    } else {
      q.tg = inb ? t : uint16_t(t & keep);
      q.keep = uint16_t(0xffff);
    }
  };
  // corrected state of one fetched value (tag tg, its phi and west/back/south phi); an
  // external point inside the box holds the immersed walls' velocity (the south box-wall
  // face of v and everything beyond the box walls hold zero)
  auto corr = [&](int fld, uint8_t tg, T val, T ph, T phx, T phz, T phy, int kind, T iyf) -> T {
    if (fld == 0) {
      const T pk = ((tg & (TAG_U | TAG_UI)) == TAG_U) ? pick : T(0);
      return (tg & TAG_U) ? val - pk - ckp * ((ph - phx) * idx) : (kind == 1 ? T(0) : ubw);
    }
    if (fld == 1) return (tg & TAG_V) ? val - ckp * ((ph - phy) * iyf) : (kind == 0 ? vbw : T(0));
    if (fld == 2) return (tg & TAG_W) ? val - ckp * ((ph - phz) * idz) : (kind == 1 ? T(0) : wbw);
    return (tg & TAG_P) ? val + ph : T(0);
  };
  // corrected state of the fetched pair into ring slot sl
  // (jj: the plane's index; beyond the box walls and on the south box-wall plane the
  // external values are zero, elsewhere the immersed walls' velocity)
  auto put = [&](int sl, int jj, const TileRaw<T>& a, bool with_phy) {
    if (has) {
      const int e = 2 * tid;   // tile index of the pair's first value
      const Pair<T> phy = with_phy ? a.phy : phprev;   // a plane outside the box has tag 0
      const uint16_t tgm = a.tg & a.keep;
      const uint8_t t0 = uint8_t(tgm & 0xff), t1 = uint8_t(tgm >> 8);
      const int kd = (jj < 0 || jj >= ny1) ? 1 : (jj == 0 ? 2 : 0);
      T iyf = idy;
      if constexpr (SY) iyf = T(g.ytab[YT_IDYF * g.ystr + min(max(jj, 0), ny1 - 1)]);
      const Pair<T> cu = {corr(0, t0, a.us.x, a.ph.x, a.phw.y, a.phz.x, phy.x, kd, iyf),
                          corr(0, t1, a.us.y, a.ph.y, a.ph.x, a.phz.y, phy.y, kd, iyf)};
      const Pair<T> cv = {corr(1, t0, a.vs.x, a.ph.x, a.phw.y, a.phz.x, phy.x, kd, iyf),
                          corr(1, t1, a.vs.y, a.ph.y, a.ph.x, a.phz.y, phy.y, kd, iyf)};
      const Pair<T> cw = {corr(2, t0, a.ws.x, a.ph.x, a.phw.y, a.phz.x, phy.x, kd, iyf),
                          corr(2, t1, a.ws.y, a.ph.y, a.ph.x, a.phz.y, phy.y, kd, iyf)};
      const Pair<T> cp = {corr(3, t0, a.pp.x, a.ph.x, a.phw.y, a.phz.x, phy.x, kd, iyf),
                          corr(3, t1, a.pp.y, a.ph.y, a.ph.x, a.phz.y, phy.y, kd, iyf)};
      *reinterpret_cast<Pair<T>*>(&ring[0][sl][e]) = cu;
      *reinterpret_cast<Pair<T>*>(&ring[1][sl][e]) = cv;
      *reinterpret_cast<Pair<T>*>(&ring[2][sl][e]) = cw;
      *reinterpret_cast<Pair<T>*>(&ring[3][sl][e]) = cp;
      phprev = a.ph;
    }
  };
  // four slots: plane j+2 goes to the slot of plane j-2, which no wave reads any more
  // once the barrier closing the previous plane has passed, so one barrier per plane
  auto slot = [](int jj) { return (jj + 4) & 3; };
  // prologue: planes j0-1, j0, j0+1 into the ring
  TileRaw<T> ha;
  {
    TileRaw<T> q0, q1, q2;
    fetch(j0 - 1, q0, true);
    fetch(j0, q1, false);
    fetch(j0 + 1, q2, false);
    put(slot(j0 - 1), j0 - 1, q0, true);
    put(slot(j0), j0, q1, false);
    put(slot(j0 + 1), j0 + 1, q2, false);
  }
  const int cc = (tz + 1) * MHX + (tx + 2);   // centre inside a tile
  __syncthreads();

  const T h = T(0.5), two = T(2), zero = T(0);
  const T idx2 = T(g.idx2), idy2 = T(g.idy2), idz2 = T(g.idz2), nu = T(g.nu);
  const T akdt = T(s.ak_dt), bkdt = T(s.bk_dt), ckdt = T(s.ck_dt);
  double qloc = 0.0;

  // Per point and plane: the tag and the list offsets of the immersed-boundary points of
  // the point's 64-wide row chunk (Ahead, loaded one plane before the coefficients that
  // they index), and the point's (B, 1/A) and held right-hand sides (PointIn).  Loads
  // complete in issue order, so each group is issued before the loads that are waited for
  // later: waiting for it does not wait for them.  With PF = 1 a plane's coefficients and
  // tile loads are issued in the plane's own iteration; with PF = 2 one iteration earlier,
  // so that every load has a whole iteration to arrive.
  struct Ahead {
    uint8_t tg;
    int cu, cv, cw;
  };
  struct PointIn {
    uint8_t tg;
    double2 cfu, cfv, cfw;
    T hu, hv, hw;
  };
  const int kc = k < nz ? k : nz - 1, icl = i < nx ? i : nx - 1;
  auto load_ahead = [&](int jj, Ahead& a) {
    const int jn = jj < ny1 ? jj : ny1 - 1;
    a.tg = f.tag[jn * plane + kc * nx + icl];
    const int ch = (jn * nz + kc) * L.cpr + chk;
    a.cu = L.choff_u[ch];
    a.cv = L.choff_v[ch];
    a.cw = L.choff_w[ch];
  };
  auto load_point = [&](int jj, const Ahead& a, PointIn& q) {
    const int jn = jj < ny1 ? jj : ny1 - 1;
    const int c = jn * plane + k * nx + i;
    const uint8_t tg = act ? a.tg : uint8_t(0);
    q.tg = tg;
    // immersed-boundary points: list index = chunk offset + flagged lanes below (the
    // wavefront is the 64-wide chunk chk of row j*nz + k); (B, 1/A) of this point
    const uint64_t mu = __ballot((tg & TAG_UI) != 0);
    const uint64_t mv = __ballot((tg & TAG_VI) != 0);
    const uint64_t mw = __ballot((tg & TAG_WI) != 0);
    const size_t cb = (size_t)s.stage * L.n_total;
    q.cfu = q.cfv = q.cfw = double2{0.0, 0.0};
    // (clamped to the list capacities: a geometry that overflowed them is reported and
    // never reads past its lists)
    if (tg & TAG_UI) q.cfu = L.coef[cb + min(a.cu + lanes_below(mu, lane), L.n_u - 1)];
    if (tg & TAG_VI) q.cfv = L.coef[cb + L.n_u + min(a.cv + lanes_below(mv, lane), L.n_v - 1)];
    if (tg & TAG_WI) q.cfw = L.coef[cb + L.n_u + L.n_v + min(a.cw + lanes_below(mw, lane), L.n_w - 1)];
    q.hu = q.hv = q.hw = T(0);
    if (act) {
      if (s.use_hold) {
        if (xcd_order & MOM_NT_LOAD) {
          q.hu = __builtin_nontemporal_load(f.Hu + c);
          q.hv = __builtin_nontemporal_load(f.Hv + c);
          q.hw = __builtin_nontemporal_load(f.Hw + c);
        } else {
          q.hu = f.Hu[c];
          q.hv = f.Hv[c];
          q.hw = f.Hw[c];
        }
      }
    }
  };
  Ahead ta, tb;
  PointIn pa, pb;
  load_ahead(j0, ta);
  if constexpr (PF == 2) {
    // the loads a loop iteration finds in flight, in the loop's own issue order
    load_point(j0, ta, pa);
    load_ahead(j0 + 1, ta);
    __builtin_amdgcn_sched_barrier(0);
    fetch(j0 + 2, ha, false);
  }
  // one plane j: the loads of the next planes are issued (point data of plane j (PF = 1)
  // or j+1 (PF = 2) into nxt with the offsets in use, offsets of the plane after that into
  // next, tile plane j+1+PF into fill) before the arithmetic of plane j; afterwards plane
  // j+2 (fill, or with PF = 2 the registers loaded one iteration earlier, hold) goes to the
  // ring
  auto plane_step = [&](int j, TileRaw<T>& hold, TileRaw<T>& fill, PointIn& cur, PointIn& nxt, Ahead& use,
                        Ahead& next) {
    const int c = j * plane + k * nx + i;
    load_point(j + PF - 1, use, nxt);
    load_ahead(j + PF, next);
    __builtin_amdgcn_sched_barrier(0);   // keep the loads above ahead of the prefetch
    fetch(j + 1 + PF, fill, false);
    const uint8_t tg = cur.tg;
    const double2 cfu = cur.cfu, cfv = cur.cfv, cfw = cur.cfw;
    const T hu = cur.hu, hv = cur.hv, hw = cur.hw;
    const T* U0 = ring[0][slot(j)];
    const T* Um = ring[0][slot(j - 1)];
    const T* Up = ring[0][slot(j + 1)];
    const T* V0 = ring[1][slot(j)];
    const T* Vm = ring[1][slot(j - 1)];
    const T* Vp = ring[1][slot(j + 1)];
    const T* W0 = ring[2][slot(j)];
    const T* Wm = ring[2][slot(j - 1)];
    const T* Wp = ring[2][slot(j + 1)];
    const T* P0 = ring[3][slot(j)];
    const T* Pm = ring[3][slot(j - 1)];
    const T uc = U0[cc], ue = U0[cc + 1], uw = U0[cc - 1], ut = U0[cc + MHX], ub = U0[cc - MHX];
    const T un = Up[cc], usb = Um[cc], u_ip_s = Um[cc + 1], u_ip_km = U0[cc - MHX + 1];
    const T vc = V0[cc], ve = V0[cc + 1], vw = V0[cc - 1], vt = V0[cc + MHX], vb = V0[cc - MHX];
    const T vn = Vp[cc], vs0 = Vm[cc], v_im_n = Vp[cc - 1], v_km_n = Vp[cc - MHX];
    const T wc = W0[cc], we = W0[cc + 1], ww = W0[cc - 1], wt = W0[cc + MHX], wb = W0[cc - MHX];
    const T wn = Wp[cc], wsb = Wm[cc], w_kp_im = W0[cc + MHX - 1], w_kp_s = Wm[cc + MHX];
    const T pc = P0[cc], pw = P0[cc - 1], pb = P0[cc - MHX], ps = Pm[cc];

    T Hu, ru, Hv, rv, Hw, rw;
    if constexpr (!SY) {
      // u-momentum at (i dx, y_c[j], z_c[k])
      {
        const T a1 = h * (uc + ue), a0 = h * (uw + uc);
        const T N = (a1 * a1 - a0 * a0) * idx +
                    (h * (uc + un) * h * (v_im_n + vn) - h * (usb + uc) * h * (vw + vc)) * idy +
                    (h * (uc + ut) * h * (w_kp_im + wt) - h * (ub + uc) * h * (ww + wc)) * idz;
        const T L = (ue - two * uc + uw) * idx2 + (un - two * uc + usb) * idy2 + (ut - two * uc + ub) * idz2;
        Hu = -N + nu * L;
        ru = akdt * Hu - ckdt * ((pc - pw) * idx);
        if (s.use_hold) ru += bkdt * hu;
      }
      // v-momentum at (x_c[i], y_f[j], z_c[k]); only stored where v is internal (j >= 1)
      {
        const T b1 = h * (vc + vn), b0 = h * (vs0 + vc);
        const T N = (h * (vc + ve) * h * (u_ip_s + ue) - h * (vw + vc) * h * (usb + uc)) * idx +
                    (b1 * b1 - b0 * b0) * idy +
                    (h * (vc + vt) * h * (w_kp_s + wt) - h * (vb + vc) * h * (wsb + wc)) * idz;
        const T L = (ve - two * vc + vw) * idx2 + (vn - two * vc + vs0) * idy2 + (vt - two * vc + vb) * idz2;
        Hv = -N + nu * L;
        rv = akdt * Hv - ckdt * ((pc - ps) * idy);
        if (s.use_hold) rv += bkdt * hv;
      }
      // w-momentum at (x_c[i], y_c[j], k dz)
      {
        const T c1 = h * (wc + wt), c0 = h * (wb + wc);
        const T N = (h * (wc + we) * h * (u_ip_km + ue) - h * (ww + wc) * h * (ub + uc)) * idx +
                    (h * (wc + wn) * h * (v_km_n + vn) - h * (wsb + wc) * h * (vb + vc)) * idy +
                    (c1 * c1 - c0 * c0) * idz;
        const T L = (we - two * wc + ww) * idx2 + (wn - two * wc + wsb) * idy2 + (wt - two * wc + wb) * idz2;
        Hw = -N + nu * L;
        rw = akdt * Hw - ckdt * ((pc - pb) * idz);
        if (s.use_hold) rw += bkdt * hw;
      }
    } else {
      // stretched wall-normal grid: per-row spacings (uniform over the block's plane),
      // three-point second derivatives with the row's own weights, u and w carried to the
      // faces by linear interpolation
      const double* yt = g.ytab;
      const int ys = g.ystr;
      const T iyc = T(yt[YT_IDYC * ys + j]), iyf = T(yt[YT_IDYF * ys + j]);
      const T dcm = T(yt[YT_DCM * ys + j]), dcp = T(yt[YT_DCP * ys + j]);
      const T dfm = T(yt[YT_DFM * ys + j]), dfp = T(yt[YT_DFP * ys + j]);
      const T wl0 = T(yt[YT_WLO * ys + j]), wh0 = T(yt[YT_WHI * ys + j]);
      const T wl1 = T(yt[YT_WLO * ys + j + 1]), wh1 = T(yt[YT_WHI * ys + j + 1]);
      {
        const T a1 = h * (uc + ue), a0 = h * (uw + uc);
        const T N = (a1 * a1 - a0 * a0) * idx +
                    ((wl1 * uc + wh1 * un) * h * (v_im_n + vn) - (wl0 * usb + wh0 * uc) * h * (vw + vc)) * iyc +
                    (h * (uc + ut) * h * (w_kp_im + wt) - h * (ub + uc) * h * (ww + wc)) * idz;
        const T L = (ue - two * uc + uw) * idx2 + (dcm * usb + dcp * un - (dcm + dcp) * uc) +
                    (ut - two * uc + ub) * idz2;
        Hu = -N + nu * L;
        ru = akdt * Hu - ckdt * ((pc - pw) * idx);
        if (s.use_hold) ru += bkdt * hu;
      }
      {
        const T b1 = h * (vc + vn), b0 = h * (vs0 + vc);
        const T N = (h * (vc + ve) * (wl0 * u_ip_s + wh0 * ue) - h * (vw + vc) * (wl0 * usb + wh0 * uc)) * idx +
                    (b1 * b1 - b0 * b0) * iyf +
                    (h * (vc + vt) * (wl0 * w_kp_s + wh0 * wt) - h * (vb + vc) * (wl0 * wsb + wh0 * wc)) * idz;
        const T L = (ve - two * vc + vw) * idx2 + (dfm * vs0 + dfp * vn - (dfm + dfp) * vc) +
                    (vt - two * vc + vb) * idz2;
        Hv = -N + nu * L;
        rv = akdt * Hv - ckdt * ((pc - ps) * iyf);
        if (s.use_hold) rv += bkdt * hv;
      }
      {
        const T c1 = h * (wc + wt), c0 = h * (wb + wc);
        const T N = (h * (wc + we) * h * (u_ip_km + ue) - h * (ww + wc) * h * (ub + uc)) * idx +
                    ((wl1 * wc + wh1 * wn) * h * (v_km_n + vn) - (wl0 * wsb + wh0 * wc) * h * (vb + vc)) * iyc +
                    (c1 * c1 - c0 * c0) * idz;
        const T L = (we - two * wc + ww) * idx2 + (dcm * wsb + dcp * wn - (dcm + dcp) * wc) +
                    (wt - two * wc + wb) * idz2;
        Hw = -N + nu * L;
        rw = akdt * Hw - ckdt * ((pc - pb) * idz);
        if (s.use_hold) rw += bkdt * hw;
      }
    }
    // single-use outputs: optionally streamed past the caches, so that the L2 keeps the
    // tile rows that neighbouring blocks load as their halos
    auto st_out = [&](T* ptr, T val) {
      if (xcd_order & MOM_NT_STORE) __builtin_nontemporal_store(val, ptr);
      else *ptr = val;
    };
    if (act) {
      if (s.write_h) {
        st_out(f.Hu + c, Hu);
        st_out(f.Hv + c, Hv);
        st_out(f.Hw + c, Hw);
      }
      // external points keep the immersed walls' velocity (v on the south box wall: 0)
      T su = ubw, sv = (j == 0) ? zero : vbw, sw = wbw;
      if (tg & TAG_U) su = uc + ru;
      if (tg & TAG_V) sv = vc + rv;
      if (tg & TAG_W) sw = wc + rw;
      // implicit IBM update (a moving wall's term sigma U_b c_k dt / A is added by the
      // flow-rate kernel, which visits the immersed-boundary points)
      if (tg & TAG_UI) su = T((cfu.x * (double)uc + (double)ru) * cfu.y);
      if (tg & TAG_VI) sv = T((cfv.x * (double)vc + (double)rv) * cfv.y);
      if (tg & TAG_WI) sw = T((cfw.x * (double)wc + (double)rw) * cfw.y);
      st_out(f.us + c, su);
      st_out(f.vs + c, sv);
      st_out(f.ws + c, sw);
      st_out(f.pn + c, pc);
      if constexpr (SY) {
        // (a uniform grid in a batched launch with stretched ones: unweighted, like its
        // flow-rate scale factor)
        if (tg & TAG_U) qloc += g.stretched ? (double)su * g.ytab[YT_DYC * g.ystr + j] : (double)su;
      } else {
        if (tg & TAG_U) qloc += (double)su;
      }
    }
    if constexpr (PF == 2) put(slot(j + 2), j + 2, hold, false);
    else put(slot(j + 2), j + 2, fill, false);
    __syncthreads();
  };
  if constexpr (PF == 2) {
    // two register sets taking turns (no copies between them, which would wait for the
    // loads in flight)
    TileRaw<T> hb;
    for (int j = j0; j < j1; j += 2) {
      plane_step(j, ha, hb, pa, pb, ta, tb);
      if (j + 1 < j1) plane_step(j + 1, hb, ha, pb, pa, tb, ta);
    }
  } else {
    for (int j = j0; j < j1; ++j) plane_step(j, ha, ha, pa, pa, ta, ta);
  }
  const double tot = block_reduce<false>(qloc, red);
  if (tid == 0) qpart[bid_x] = tot;
}

template <typename T, bool SY, int MXT, int MZT, int PF = 1>
__global__ __launch_bounds__(MXT * MZT) void k_momentum(GridParams g, Fields<T> f, IbmLists L, StageConsts s, int jc,
                                                 int ntx, int ntz, int xcd_order, const double* __restrict__ pi_prev,
                                                 double ckdt_prev, double* __restrict__ qpart) {
  k_momentum_body<T, SY, MXT, MZT, PF>(g, f, L, s, jc, ntx, ntz, xcd_order, pi_prev, ckdt_prev, qpart, blockIdx.x,
                                   blockIdx.y, gridDim.x);
}

// The same for a batch of independent grids in one launch (block ranges boff); in FP64
// held to 168 registers, 3 waves per SIMD like the single-grid kernel (170 without the
// bound, which left 2).
template <typename T, bool SY>
__global__ __launch_bounds__(256, sizeof(T) == 8 && !SY ? 3 : 1) void k_momentum_b(const MomArgs<T>* __restrict__ args,
    const int* __restrict__ boff, int ninst) {
  const int i = batch_instance(boff, ninst, blockIdx.x);
  const MomArgs<T>& a = args[i];
  const int local = blockIdx.x - boff[i];
  k_momentum_body<T, SY>(a.g, a.f, a.L, a.s, a.jc, a.ntx, a.ntz, a.xcd_order, a.pi_prev, a.ckdt_prev, a.qpart, local % a.gx, local / a.gx, boff[i + 1] - boff[i]);
}

// ---------------------------------------------------------------------------------------
// cfr_pi: Q(u*_0) = (dy dz / nx) sum u*_0 over internal u; Pi_k = (Q - Q_t) / S_k so that
// Q(u*_0 - Pi_k c_k dt / A) = Q_t exactly (constant pressure gradient: Pi_k = Pi).  Every
// block reduces the momentum partials in the same fixed order (so all blocks hold the
// same Pi_k, deterministically); block 0 publishes it for the later kernels; each thread
// applies u* -= Pi_k c_k dt / A at one immersed-boundary u face.  div_fftx, correct and
// the diagnostics apply -Pi_k c_k dt to the other internal u faces themselves.
// ---------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void k_cfr_pi_body(Fields<T> f, IbmLists L, int stage, double ck_dt,
                                               const double* __restrict__ qpart, int nq, double scale, int forcing,
                                               double qt, const double* __restrict__ S3,
                                               double* __restrict__ pi_out, double* __restrict__ pi_hist, int bid_x, int bid_y, int nblk) {
  __shared__ double red[4];
  __shared__ double pi_s;
  // this thread's immersed-boundary point (a u face; with moving walls any component) and
  // its predictor are loaded first, so that their latency overlaps the reduction
  const int g = bid_x * blockDim.x + threadIdx.x;
  int id = 0;
  double inva = 0.0, usv = 0.0, add = 0.0;
  T* fp = f.us;
  // entry g of the capacity-strided lists holds a point if it is below its component's count
  const int comp = g < L.n_u ? 0 : (g < L.n_u + L.n_v ? 1 : 2);
  const int coff = comp == 0 ? 0 : (comp == 1 ? L.n_u : L.n_u + L.n_v);
  const int ccap = comp == 0 ? L.n_u : (comp == 1 ? L.n_v : L.n_w);
  const bool pt = g < L.n_cover && g - coff < min(L.cnt[comp], ccap);
  if (pt) {
    fp = comp == 0 ? f.us : (comp == 1 ? f.vs : f.ws);
    id = L.idx[g];
    inva = L.coef[(size_t)stage * L.n_total + g].y;
    usv = (double)fp[id];
    // a moving wall's term sigma U_b c_k dt / A of the implicit update (zero at rest)
    add = L.sig[g] * ck_dt * L.wallv[comp] * inva;
  }
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int stride = blockDim.x * 8;
  for (int base = threadIdx.x; base < nq; base += stride) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int e = base + r * blockDim.x;
      if (e < nq) acc[r] += qpart[e];
    }
  }
  const double s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  const double tot = block_reduce<false>(s, red);
  if (threadIdx.x == 0) {
    // the partials hold u* without the moving walls' term; its sum over the IBM u points
    // is c_k dt U_b sum(sig / A)
    const double q0 = (tot + ck_dt * L.wallv[0] * L.sd[stage]) * scale;
    const double pi = (forcing == 0) ? (q0 - qt) / S3[stage] : qt;
    pi_s = pi;
    if (bid_x == 0) {
      pi_out[0] = pi;
      pi_hist[0] = pi;
      pi_hist[1] = q0;
    }
  }
  __syncthreads();
  if (pt) fp[id] = T(usv + add - (g < L.n_u ? pi_s * ck_dt * inva : 0.0));
}

template <typename T>
__global__ __launch_bounds__(256) void k_cfr_pi(Fields<T> f, IbmLists L, int stage, double ck_dt,
                                               const double* __restrict__ qpart, int nq, double scale, int forcing,
                                               double qt, const double* __restrict__ S3,
                                               double* __restrict__ pi_out, double* __restrict__ pi_hist) {
  k_cfr_pi_body<T>(f, L, stage, ck_dt, qpart, nq, scale, forcing, qt, S3, pi_out, pi_hist, blockIdx.x, blockIdx.y, gridDim.x);
}

// The same for a batch of independent grids in one launch (block ranges boff).
template <typename T>
__global__ __launch_bounds__(256) void k_cfr_pi_b(const CfrArgs<T>* __restrict__ args,
    const int* __restrict__ boff, int ninst) {
  const int i = batch_instance(boff, ninst, blockIdx.x);
  const CfrArgs<T>& a = args[i];
  const int local = blockIdx.x - boff[i];
  k_cfr_pi_body<T>(a.f, a.L, a.stage, a.ck_dt, a.qpart, a.nq, a.scale, a.forcing, a.qt, a.S3, a.pi_out, a.pi_hist, local % a.gx, local / a.gx, boff[i + 1] - boff[i]);
}

// ---------------------------------------------------------------------------------------
// div_fftx: rhs = D u* / (c_k dt) on every cell, then the real FFT along x of each
// (j, k) row: the nx reals are packed as nx/2 complex numbers z_n = x_{2n} + i x_{2n+1},
// transformed, and unpacked to X_m, m = 0..nx/2.  2^ll lanes per row (as few as keep
// every FFT stage at one butterfly per lane), blockDim.x >> ll rows per block.
// If rhs_in is given, it replaces the divergence (stand-alone Poisson solve).
// ---------------------------------------------------------------------------------------
template <typename T, int MB>
__device__ __forceinline__ void k_div_fftx_body(GridParams g, Fields<T> f, IbmLists L, int stage, FFTPlan px,
                                                 const double2* __restrict__ rtw, double ck_dt,
                                                 const double* __restrict__ pi, const T* __restrict__ rhs_in, int ll,
                                                 int bid_x, int bid_y, int nblk) {
  if (g.skip && *g.skip) return;   // a converged masked solve: nothing left to do
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* sm = reinterpret_cast<cplx<T>*>(smem_raw);
  const int N = g.nhalf;
  const int RB = blockDim.x >> ll;             // rows per block
  const int NL = 1 << ll;                      // lanes per row
  const int grp = threadIdx.x >> ll, lane = threadIdx.x & (NL - 1);
  const int row = bid_x * RB + grp;
  const int nx = g.nx;
  cplx<T>* A = sm + grp * N;
  cplx<T>* tw = sm + RB * N;
  load_twiddles<T>(tw, px, threadIdx.x, blockDim.x);
  const bool valid = row < g.nrows;
  if (valid) {
    // each lane takes pairs of x-adjacent points (one vector load per field), which are
    // also the packed complex values z_n = x_{2n} + i x_{2n+1}
    const int rb = row * nx;
    if (rhs_in) {   // a caller's array: element loads, no alignment assumed
      for (int n = lane; n < N; n += NL) A[n] = cplx<T>{rhs_in[rb + 2 * n], rhs_in[rb + 2 * n + 1]};
    } else {
      const int j = row / g.nz, k = row - (row / g.nz) * g.nz;
      const int kp = wrap_p(k, g.nz);
      const T pick = T(pi[0] * ck_dt);
      const T inv = T(1.0 / ck_dt);
      const T idx = T(g.idx), idz = T(g.idz);
      const T idy = T(g.stretched ? g.ytab[YT_IDYC * g.ystr + j] : g.idy);
      const bool hasN = (j + 1 < g.ny1);
      const int plane = nx * g.nz;
      // u* on a u face: internal non-IBM faces still owe -Pi c_k dt (= pick)
      auto ust = [&](T u, uint8_t tg) { return u - (((tg & (TAG_U | TAG_UI)) == TAG_U) ? pick : T(0)); };
      for (int n = lane; n < N; n += NL) {
        const int c = rb + 2 * n;
        const int ie = rb + (2 * n + 2 == nx ? 0 : 2 * n + 2);   // east of the pair's second point
        const Pair<T> u2 = ld_pair(f.us + c);
        const T u3 = f.us[ie];
        const uint16_t t2 = *reinterpret_cast<const uint16_t*>(f.tag + c);
        const uint8_t t3 = f.tag[ie];
        const Pair<T> vc2 = ld_pair(f.vs + c);
        const Pair<T> vn2 = hasN ? ld_pair(f.vs + c + plane) : Pair<T>{T(0), T(0)};
        const Pair<T> wc2 = ld_pair(f.ws + c);
        const Pair<T> wt2 = ld_pair(f.ws + c + (kp - k) * nx);
        const T a0 = ust(u2.x, uint8_t(t2 & 0xff)), a1 = ust(u2.y, uint8_t(t2 >> 8)), a2 = ust(u3, t3);
        A[n] = cplx<T>{((a1 - a0) * idx + (vn2.x - vc2.x) * idy + (wt2.x - wc2.x) * idz) * inv,
                       ((a2 - a1) * idx + (vn2.y - vc2.y) * idy + (wt2.y - wc2.y) * idz) * inv};
      }
    }
  }
  __syncthreads();
  fft_lds<T, MB>(A, 0, px, tw, -1, lane, NL);
  const cplx<T>* R = A;
  if (valid) {
    const int jr = row / g.nz;
    cplx<T>* out = f.spec + (size_t)jr * g.splane + (size_t)(row - jr * g.nz) * g.mhs;
    // modes m and N - m from the same two values: X_{N-m} takes the twiddle
    // e^{-2 pi i (N-m)/nx} = -conj(e^{-2 pi i m/nx}); m = 0 also gives X_N
    for (int m = lane; m <= N / 2; m += NL) {
      const cplx<T> Zm = R[m], Zn = R[m == 0 ? 0 : N - m];
      const double2 e64 = rtw[m];
      const cplx<T> e = {T(e64.x), T(e64.y)};
      {
        const cplx<T> Zc = cconj(Zn);
        const cplx<T> s1 = cadd(Zm, Zc), d1 = csub(Zm, Zc);
        const cplx<T> t = cmul(e, d1);
        out[m] = cplx<T>{T(0.5) * (s1.x + t.y), T(0.5) * (s1.y - t.x)};
      }
      if (2 * m != N) {
        const cplx<T> Zc = cconj(Zm);
        const cplx<T> s1 = cadd(Zn, Zc), d1 = csub(Zn, Zc);
        const cplx<T> t = cmul(cplx<T>{-e.x, e.y}, d1);
        out[N - m] = cplx<T>{T(0.5) * (s1.x + t.y), T(0.5) * (s1.y - t.x)};
      }
    }
  }
}

template <typename T, int MB>
__global__ __launch_bounds__(256) void k_div_fftx(GridParams g, Fields<T> f, IbmLists L, int stage, FFTPlan px,
                                                 const double2* __restrict__ rtw, double ck_dt,
                                                 const double* __restrict__ pi, const T* __restrict__ rhs_in,
                                                 int ll) {
  k_div_fftx_body<T, MB>(g, f, L, stage, px, rtw, ck_dt, pi, rhs_in, ll, blockIdx.x, blockIdx.y, gridDim.x);
}

// The same for a batch of independent grids in one launch (block ranges boff).
template <typename T, int MB>
__global__ __launch_bounds__(256) void k_div_fftx_b(const DivArgs<T>* __restrict__ args,
    const int* __restrict__ boff, int ninst) {
  const int i = batch_instance(boff, ninst, blockIdx.x);
  const DivArgs<T>& a = args[i];
  const int local = blockIdx.x - boff[i];
  k_div_fftx_body<T, MB>(a.g, a.f, a.L, a.stage, a.px, a.rtw, a.ck_dt, a.pi, a.rhs_in, a.ll, local % a.gx, local / a.gx, boff[i + 1] - boff[i]);
}

// ---------------------------------------------------------------------------------------
// fftz: complex FFT along z of the half spectrum, W columns (one x mode m of one plane j)
// at a time per block.  The first blocks take W consecutive modes of NJ consecutive
// planes, one plane after the other; with RP > 0 the next plane's columns are loaded into
// registers (RP values per thread) while the current one is transformed and stored.  The
// mh mod W modes left over at the end of every plane are gathered, W at a time, into the
// last blocks (one plane each), so that no block transforms padding columns.
// ---------------------------------------------------------------------------------------
template <typename T, int MB, int RP>
__device__ __forceinline__ void k_fftz_body(GridParams g, cplx<T>* __restrict__ spec, FFTPlan pz, int sign,
                                             int W, int NJ, int b) {
  if (g.skip && *g.skip) return;   // a converged masked solve: nothing left to do
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* A = reinterpret_cast<cplx<T>*>(smem_raw);
  const int nz = g.nz, mh = g.mh, mhs = g.mhs;
  cplx<T>* tw = A + nz * W;
  load_twiddles<T>(tw, pz, threadIdx.x, blockDim.x);
  const int lw = __ffs(W) - 1;   // W is a power of two
  const int w = threadIdx.x & (W - 1), lane = threadIdx.x >> lw, nl = blockDim.x >> lw;
  const int gxf = mh >> lw, rem = mh - (gxf << lw);
  const int nfull = gxf * ((g.ny1 + NJ - 1) / NJ);
  if (b < nfull) {
    const int jb = b / gxf;
    const int m = ((b - jb * gxf) << lw) + w;
    const int ja = jb * NJ, je = min(ja + NJ, g.ny1);
    if (RP > 0) {
      T prx[RP > 0 ? RP : 1], pry[RP > 0 ? RP : 1];   // next plane's values (re, im)
      {
        const cplx<T>* col = spec + (size_t)ja * g.splane + m;
#pragma unroll
        for (int r = 0; r < RP; ++r) {
          const int kz = min(lane + r * nl, nz - 1);   // clamped: a repeated load is never stored
          const cplx<T> v = col[(size_t)kz * mhs];
          prx[r] = v.x;
          pry[r] = v.y;
        }
      }
      for (int j = ja; j < je; ++j) {
#pragma unroll
        for (int r = 0; r < RP; ++r) {
          const int kz = lane + r * nl;
          if (kz < nz) A[(kz << lw) + w] = cplx<T>{prx[r], pry[r]};
        }
        __syncthreads();
        if (j + 1 < je) {   // the next plane's loads are in flight during this plane's transform and store
          const cplx<T>* col = spec + (size_t)(j + 1) * g.splane + m;
#pragma unroll
          for (int r = 0; r < RP; ++r) {
            const int kz = min(lane + r * nl, nz - 1);
            const cplx<T> v = col[(size_t)kz * mhs];
            prx[r] = v.x;
            pry[r] = v.y;
          }
        }
        fft_lds<T, MB>(A + w, lw, pz, tw, sign, lane, nl);
        cplx<T>* col = spec + (size_t)j * g.splane + m;
        for (int kz = lane; kz < nz; kz += nl) col[(size_t)kz * mhs] = A[(kz << lw) + w];
        __syncthreads();   // the next plane overwrites A
      }
    } else {
      for (int j = ja; j < je; ++j) {
        cplx<T>* col = spec + (size_t)j * g.splane + m;   // element kz at col[kz * mhs]
        for (int kz = lane; kz < nz; kz += nl) A[(kz << lw) + w] = col[(size_t)kz * mhs];
        __syncthreads();
        fft_lds<T, MB>(A + w, lw, pz, tw, sign, lane, nl);
        for (int kz = lane; kz < nz; kz += nl) col[(size_t)kz * mhs] = A[(kz << lw) + w];
        __syncthreads();
      }
    }
    return;
  }
  // a remainder block: this thread's column (plane j, mode m)
  const int idx = ((b - nfull) << lw) + w;
  const bool ok = rem > 0 && idx < rem * g.ny1;
  int j = 0, m = 0;
  if (ok) {
    j = idx / rem;
    m = (gxf << lw) + idx - j * rem;
  }
  cplx<T>* col = spec + (size_t)j * g.splane + m;   // element kz at col[kz * mhs]
  for (int kz = lane; kz < nz; kz += nl) A[(kz << lw) + w] = ok ? col[(size_t)kz * mhs] : cplx<T>{T(0), T(0)};
  __syncthreads();
  fft_lds<T, MB>(A + w, lw, pz, tw, sign, lane, nl);
  if (ok)
    for (int kz = lane; kz < nz; kz += nl) col[(size_t)kz * mhs] = A[(kz << lw) + w];
}

template <typename T, int MB, int RP>
__global__ __launch_bounds__(512) void k_fftz(GridParams g, cplx<T>* __restrict__ spec, FFTPlan pz, int sign,
                                             int W, int NJ) {
  k_fftz_body<T, MB, RP>(g, spec, pz, sign, W, NJ, blockIdx.x);
}

// The same for a batch of independent grids in one launch (block ranges boff), a.nj
// planes per full block (several, with the next plane held in RP registers per thread,
// when every instance's share of a column fits them).
template <typename T, int MB, int RP>
__global__ __launch_bounds__(512) void k_fftz_b(const FftzArgs<T>* __restrict__ args,
    const int* __restrict__ boff, int ninst) {
  const int i = batch_instance(boff, ninst, blockIdx.x);
  const FftzArgs<T>& a = args[i];
  const int local = blockIdx.x - boff[i];
  k_fftz_body<T, MB, RP>(a.g, a.spec, a.pz, a.sign, a.W, a.nj, local);
}

// ---------------------------------------------------------------------------------------
// tri: per Fourier mode (kx, kz), solve in y
//   (phi_{j+1} - 2 phi_j + phi_{j-1}) / dy^2 - (kx^2 + kz^2) phi_j = rhat_j / (nx nz)
// with -1 instead of -2 in the first and last rows (no flux through the box walls).
// Mode (0,0): its mean over j is removed, the first row becomes phi_0 = 0, and the
// mean of the solution is removed.
//
// Partition (divide-and-conquer) solver, FP64 arithmetic in registers and LDS:
// P threads per mode each own a segment of L <= 8 consecutive rows.  Within its
// segment a thread eliminates the sub-diagonal downwards and the super-diagonal
// upwards, leaving every interior unknown expressed through the segment's first (F)
// and last (E) unknowns.  The 2P equations of the F and E unknowns form a
// tridiagonal system (ordered F0 E0 F1 E1 ...) solved by parallel cyclic reduction
// in LDS; each thread then recovers its interior rows.  The spectrum is read once
// and written once.  W = 256/P modes per block, lane = p * W + w.
// ---------------------------------------------------------------------------------------
// Row stride (in doubles) of the reduced-system arrays.  A wavefront holds 64 / W segment
// groups of W modes (8W bytes each) at a stride of two rows; with W a power of two up to
// 16 the stride is 3W/2, so that the stride over a group's bytes is odd and successive
// groups fall on different LDS banks (a stride of W put every group on the same half of
// the banks); other W keep W padded to 8 modulo 16.
__host__ __device__ inline int tri_rs(int W) {
  if (W >= 2 && W <= 16 && (W & (W - 1)) == 0) return 3 * W / 2;
  return W + ((8 - W % 16) + 16) % 16;
}

template <typename T, int LM, bool SY>
__device__ __forceinline__ void k_tri_body(GridParams g, cplx<T>* __restrict__ spec,
                                            const double* __restrict__ kx2, const double* __restrict__ kz2,
                                            int P, int W, double* __restrict__ mean_out, int bid_x, int gather) {
  if (g.skip && *g.skip) return;   // a converged masked solve: nothing left to do
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lds = reinterpret_cast<double*>(smem_raw);
  const int n = g.ny1;
  const int tid = threadIdx.x;
  const int p = tid / W, w = tid - p * W;
  const bool active = p < P;
  // modes.  Without gather: W consecutive entries of the spectrum order kz*mhs + m per
  // block (aligned runs), the rows' padding entries skipped.  With gather (rows with much
  // padding): the mh mod W modes left over at the end of every z row, W at a time, in the
  // first blocks (their scattered accesses overlap with the rest of the grid), then W
  // consecutive modes of one row per block.  zb: the block holding mode (0, 0), at w = 0.
  int kz, m, zb = 0;
  bool mode_ok;
  if (!gather) {
    const int q = bid_x * W + w;
    kz = q / g.mhs;
    m = q - kz * g.mhs;
    mode_ok = kz < g.nz && m < g.mh;
  } else {
    const int gpr = g.mh / W, rem = g.mh - gpr * W, nremb = (rem * g.nz + W - 1) / W;
    zb = gpr > 0 ? nremb : 0;
    if (bid_x < nremb) {
      const int idx = bid_x * W + w;
      mode_ok = idx < rem * g.nz;
      kz = mode_ok ? idx / rem : 0;
      m = gpr * W + (mode_ok ? idx - kz * rem : 0);
    } else {
      const int b = bid_x - nremb;
      kz = b / gpr;
      m = (b - kz * gpr) * W + w;
      mode_ok = true;
    }
  }
  const int qa = kz * g.mhs + m;
  const bool valid = active && mode_ok;
  const int r0 = (p * n) / P;   // p n < 2^31 (p <= 256, n < 2049)
  const int r1 = active ? ((p + 1) * n) / P : r0;
  const int L = r1 - r0;
  const double a = g.idy2;
  const double norm = 1.0 / ((double)g.nx * (double)g.nz);
  const int N2 = 2 * P;
  const int RS = tri_rs(W);
  double* Rl = lds;                 // [2P][RS] reduced system (mode fastest), unit diagonal
  double* Ru = Rl + RS * N2;
  double* Rr = Ru + RS * N2;
  double* Ri = Rr + RS * N2;
  double* red = Ri + RS * N2;       // [2P] sums of the (0,0) mode
  const double K2 = valid ? kx2[m] + kz2[kz] : 0.0;
  const bool zmode = valid && qa == 0;
  double dr[LM], di[LM];
#pragma unroll
  for (int t = 0; t < LM; ++t) {
    dr[t] = 0.0;
    di[t] = 0.0;
    if (valid && t < L) {
      const cplx<T> v = spec[(size_t)(r0 + t) * g.splane + qa];
      dr[t] = (double)v.x;
      di[t] = (double)v.y;
    }
  }
  // mean of the (0,0) mode over j (only block zb holds it, at w = 0); on a stretched grid
  // weighted by the cell heights (entry ny1 of their table holds the box height)
  constexpr bool sy = SY;
  const double* yt = g.ytab;
  const int ys = g.ystr;
  double mr = 0.0, mi = 0.0;
  if (bid_x == zb) {
    if (w == 0 && active) {
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int t = 0; t < LM; ++t)
        if (t < L) {
          const double wt = sy ? yt[YT_DYC * ys + r0 + t] : 1.0;
          sr += sy ? dr[t] * wt : dr[t];
          si += sy ? di[t] * wt : di[t];
        }
      red[p] = sr;
      red[P + p] = si;
    }
    __syncthreads();
    if (w == 0) {
      for (int pp = 0; pp < P; ++pp) { mr += red[pp]; mi += red[P + pp]; }
      const double den = sy ? yt[YT_DYC * ys + n] : (double)n;
      mr /= den;
      mi /= den;
      if (tid == 0) mean_out[0] = mr * norm;
    }
    __syncthreads();
  }
  // Row coefficients: interior rows have (a, -2a - K2, a).  The box's first row has no
  // lower coefficient and a diagonal raised by a (for the (0,0) mode it becomes phi_0 = 0:
  // diagonal 1, no upper coefficient); the box's last row has no upper coefficient and a
  // diagonal raised by a.  Segments hold L >= 2 rows, so the first row can only be a
  // segment's row 0 and the last row only its row L-1.
  const bool first = r0 == 0, last = r1 == n;
  const double dI = -2.0 * a - K2, dLast = dI + a;
  // coefficients of segment row t: lower, upper and (t >= 1) diagonal; a stretched grid
  // takes its per-row values (the box's last row has no upper coefficient)
  auto lo_ = [&](int t) -> double { return sy ? yt[YT_TLO * ys + r0 + t] : a; };
  auto hi_ = [&](int t) -> double { return sy ? yt[YT_THI * ys + r0 + t] : a; };
  auto dg_ = [&](int t, bool boxlast) -> double {
    if (sy) return boxlast ? -lo_(t) - K2 : -(lo_(t) + hi_(t)) - K2;
    return boxlast ? dLast : dI;
  };
#pragma unroll
  for (int t = 0; t < LM; ++t) {
    dr[t] = (dr[t] - mr) * norm;
    di[t] = (di[t] - mi) * norm;
  }
  if (zmode && r0 == 0) { dr[0] = 0.0; di[0] = 0.0; }
  // downward elimination: rows t >= 1 become al[t] x0 + be[t] x_t + up x_{t+1} = d_t;
  // ib[t] = 1 / be[t] also serves the upward sweep and the back substitution
  double al[LM], ib[LM], ga[LM];
#pragma unroll
  for (int t = 0; t < LM; ++t) { al[t] = 0.0; ib[t] = 1.0; ga[t] = 0.0; }
  if (valid) {
    al[1] = lo_(1);
    ib[1] = recip(dg_(1, last && L == 2));
#pragma unroll
    for (int t = 2; t < LM; ++t) {
      if (t < L) {
        const double m = lo_(t) * ib[t - 1];
        al[t] = -m * al[t - 1];
        ib[t] = recip(dg_(t, last && t == L - 1) - m * hi_(t - 1));
        dr[t] -= m * dr[t - 1];
        di[t] -= m * di[t - 1];
      }
    }
    // upward elimination: rows 1..L-2 become al[t] x0 + be[t] x_t + ga[t] x_{L-1} = d_t
    if (L >= 3) {
#pragma unroll
      for (int t = 1; t < LM; ++t)
        if (t == L - 2) ga[t] = hi_(t);
#pragma unroll
      for (int t = LM - 3; t >= 1; --t) {
        if (t <= L - 3) {
          const double m = hi_(t) * ib[t + 1];
          al[t] -= m * al[t + 1];
          ga[t] = -m * ga[t + 1];
          dr[t] -= m * dr[t + 1];
          di[t] -= m * di[t + 1];
        }
      }
    }
    // reduced equations of F = x_0 and E = x_{L-1} (segments hold L >= 2 rows), each
    // divided by its diagonal
    const int eF = (2 * p) * RS + w, eE = eF + RS;
    double dL = dr[0], dLi = di[0], alL = 0.0, ibL = 1.0, hiL = a;
#pragma unroll
    for (int t = 1; t < LM; ++t)
      if (t == L - 1) { dL = dr[t]; dLi = di[t]; alL = al[t]; ibL = ib[t]; hiL = hi_(t); }
    Rl[eE] = alL * ibL;
    Ru[eE] = last ? 0.0 : hiL * ibL;
    Rr[eE] = dL * ibL;
    Ri[eE] = dLi * ibL;
    const bool pin = zmode && first;   // phi_0 = 0 of the (0,0) mode
    double dF = pin ? 1.0 : (sy ? (first ? -hi_(0) - K2 : -(lo_(0) + hi_(0)) - K2) : (first ? dI + a : dI));
    double uF = pin ? 0.0 : hi_(0), rF = dr[0], iF = di[0];
    if (L >= 3) {
      const double m = uF * ib[1];
      dF -= m * al[1];
      uF = -m * ga[1];
      rF -= m * dr[1];
      iF -= m * di[1];
    }
    const double idF = recip(dF);
    Rl[eF] = first ? 0.0 : lo_(0) * idF;
    Ru[eF] = uF * idF;
    Rr[eF] = rF * idF;
    Ri[eF] = iF * idF;
  }
  __syncthreads();
  // Parallel cyclic reduction of the reduced system: each thread owns rows 2p and 2p+1 of
  // its mode; at stride s every row eliminates its couplings to rows e-s and e+s and is
  // divided by its new diagonal, so the right-hand side ends as the solution.
  for (int st = 1; st < N2; st <<= 1) {
    double nl[2], nu[2], nr[2], ni[2];
    if (valid) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int e = 2 * p + h;
        const int ie = e * RS + w;
        const double l = Rl[ie], u = Ru[ie];
        double r = Rr[ie], im = Ri[ie], d = 1.0, l2 = 0.0, u2 = 0.0;
        if (e - st >= 0) {
          const int j = (e - st) * RS + w;
          l2 = -l * Rl[j];
          d -= l * Ru[j];
          r -= l * Rr[j];
          im -= l * Ri[j];
        }
        if (e + st < N2) {
          const int j = (e + st) * RS + w;
          u2 = -u * Ru[j];
          d -= u * Rl[j];
          r -= u * Rr[j];
          im -= u * Ri[j];
        }
        const double id = recip(d);
        nl[h] = l2 * id; nu[h] = u2 * id; nr[h] = r * id; ni[h] = im * id;
      }
    }
    __syncthreads();
    if (valid) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int ie = (2 * p + h) * RS + w;
        Rl[ie] = nl[h]; Ru[ie] = nu[h]; Rr[ie] = nr[h]; Ri[ie] = ni[h];
      }
    }
    __syncthreads();
  }
  double xr_[LM], xi_[LM];
  if (valid) {
    const int eF = (2 * p) * RS + w, eE = eF + RS;
    const double Fr = Rr[eF], Fi = Ri[eF], Er = Rr[eE], Ei = Ri[eE];
#pragma unroll
    for (int t = 0; t < LM; ++t) {
      xr_[t] = (dr[t] - al[t] * Fr - ga[t] * Er) * ib[t];
      xi_[t] = (di[t] - al[t] * Fi - ga[t] * Ei) * ib[t];
      if (t == 0) { xr_[t] = Fr; xi_[t] = Fi; }
      if (t == L - 1) { xr_[t] = Er; xi_[t] = Ei; }
    }
  }
  // remove the mean of the (0,0) solution
  if (bid_x == zb) {
    __syncthreads();
    if (w == 0 && active) {
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int t = 0; t < LM; ++t)
        if (t < L) { sr += xr_[t]; si += xi_[t]; }
      red[p] = sr;
      red[P + p] = si;
    }
    __syncthreads();
    if (zmode) {
      double sr = 0.0, si = 0.0;
      for (int pp = 0; pp < P; ++pp) { sr += red[pp]; si += red[P + pp]; }
      sr /= n;
      si /= n;
#pragma unroll
      for (int t = 0; t < LM; ++t) { xr_[t] -= sr; xi_[t] -= si; }
    }
  }
  if (valid) {
#pragma unroll
    for (int t = 0; t < LM; ++t)
      if (t < L) spec[(size_t)(r0 + t) * g.splane + qa] = cplx<T>{T(xr_[t]), T(xi_[t])};
  }
}

// Whether the tridiagonal blocks gather the modes left over at the end of the z rows
// (rows with more than 5 % padding), and the blocks of one launch of W modes each.
__host__ __device__ inline int tri_gather(const GridParams& g) { return (g.mhs - g.mh) * 20 > g.mhs ? 1 : 0; }
__host__ __device__ inline int tri_blocks(const GridParams& g, int W, int gather) {
  if (!gather) return (g.nz * g.mhs + W - 1) / W;
  const int gpr = g.mh / W, rem = g.mh - gpr * W;
  return gpr * g.nz + (rem * g.nz + W - 1) / W;
}

template <typename T, int LM, bool SY>
__global__ __launch_bounds__(256) void k_tri(GridParams g, cplx<T>* __restrict__ spec,
                                            const double* __restrict__ kx2, const double* __restrict__ kz2,
                                            int P, int W, double* __restrict__ mean_out, int gather) {
  k_tri_body<T, LM, SY>(g, spec, kx2, kz2, P, W, mean_out, blockIdx.x, gather);
}

// The same for a batch of independent grids in one launch (block ranges boff).
template <typename T, int LM, bool SY>
__global__ __launch_bounds__(256) void k_tri_b(const TriArgs<T>* __restrict__ args,
    const int* __restrict__ boff, int ninst) {
  const int i = batch_instance(boff, ninst, blockIdx.x);
  const TriArgs<T>& a = args[i];
  const int local = blockIdx.x - boff[i];
  k_tri_body<T, LM, SY>(a.g, a.spec, a.kx2, a.kz2, a.P, a.W, a.mean_out, local, a.gather);
}

// ---------------------------------------------------------------------------------------
// ifftx: inverse real FFT along x of each row: Z_m = (X_m + conj X_{N-m})
//        + i e^{+2 pi i m/nx} (X_m - conj X_{N-m}), m < N = nx/2, z = IDFT_N(Z),
//        x_{2n} = Re z_n, x_{2n+1} = Im z_n.  Unnormalised (tri applied 1/(nx nz)).
// ---------------------------------------------------------------------------------------
template <typename T, int MB>
__device__ __forceinline__ void k_ifftx_body(GridParams g, const cplx<T>* __restrict__ spec, T* __restrict__ out,
                                              FFTPlan px, const double2* __restrict__ rtw, int ll, int bid_x, int bid_y, int nblk) {
  if (g.skip && *g.skip) return;   // a converged masked solve: nothing left to do
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* sm = reinterpret_cast<cplx<T>*>(smem_raw);
  const int N = g.nhalf;
  const int RB = blockDim.x >> ll;             // rows per block
  const int NL = 1 << ll;                      // lanes per row
  const int grp = threadIdx.x >> ll, lane = threadIdx.x & (NL - 1);
  const int row = bid_x * RB + grp;
  cplx<T>* A = sm + grp * N;
  cplx<T>* tw = sm + RB * N;
  load_twiddles<T>(tw, px, threadIdx.x, blockDim.x);
  const bool valid = row < g.nrows;
  if (valid) {
    const int jr = row / g.nz;
    const cplx<T>* in = spec + (size_t)jr * g.splane + (size_t)(row - jr * g.nz) * g.mhs;
    // modes m and N - m from the same two loads: Z_{N-m} takes the twiddle
    // e^{+2 pi i (N-m)/nx} = -conj(e^{+2 pi i m/nx})
    for (int m = lane; m <= N / 2; m += NL) {
      const cplx<T> X = in[m], Y = in[N - m];
      const double2 e64 = rtw[m];
      const cplx<T> e = {T(e64.x), T(-e64.y)};   // e^{+2 pi i m / nx}
      {
        const cplx<T> Yc = cconj(Y);
        const cplx<T> s1 = cadd(X, Yc), d1 = csub(X, Yc);
        const cplx<T> t = cmul(e, d1);
        A[m] = cplx<T>{s1.x - t.y, s1.y + t.x};
      }
      if (m > 0 && 2 * m != N) {
        const cplx<T> Xc = cconj(X);
        const cplx<T> s1 = cadd(Y, Xc), d1 = csub(Y, Xc);
        const cplx<T> t = cmul(cplx<T>{-e.x, e.y}, d1);
        A[N - m] = cplx<T>{s1.x - t.y, s1.y + t.x};
      }
    }
  }
  __syncthreads();
  fft_lds<T, MB>(A, 0, px, tw, +1, lane, NL);
  const cplx<T>* R = A;
  if (valid) {
    T* orow = out + (size_t)row * g.nx;   // x_{2n}, x_{2n+1} = Re, Im z_n
    if ((reinterpret_cast<uintptr_t>(out) & (2 * sizeof(T) - 1)) == 0) {   // one vector store per pair
      Pair<T>* o2 = reinterpret_cast<Pair<T>*>(orow);
      for (int n = lane; n < N; n += NL) o2[n] = Pair<T>{R[n].x, R[n].y};
    } else {   // a caller's array that is not pair-aligned
      for (int n = lane; n < N; n += NL) {
        orow[2 * n] = R[n].x;
        orow[2 * n + 1] = R[n].y;
      }
    }
  }
}

template <typename T, int MB>
__global__ __launch_bounds__(256) void k_ifftx(GridParams g, const cplx<T>* __restrict__ spec, T* __restrict__ out,
                                              FFTPlan px, const double2* __restrict__ rtw, int ll) {
  k_ifftx_body<T, MB>(g, spec, out, px, rtw, ll, blockIdx.x, blockIdx.y, gridDim.x);
}

// The same for a batch of independent grids in one launch (block ranges boff).
template <typename T, int MB>
__global__ __launch_bounds__(256) void k_ifftx_b(const IfftxArgs<T>* __restrict__ args,
    const int* __restrict__ boff, int ninst) {
  const int i = batch_instance(boff, ninst, blockIdx.x);
  const IfftxArgs<T>& a = args[i];
  const int local = blockIdx.x - boff[i];
  k_ifftx_body<T, MB>(a.g, a.spec, a.out, a.px, a.rtw, a.ll, local % a.gx, local / a.gx, boff[i + 1] - boff[i]);
}

// ---------------------------------------------------------------------------------------
// correct: the state after a projection (corrected_point: u = u* - c_k dt G phi on
// internal faces, the pending -Pi c_k dt included, the walls' velocity on external faces;
// p = p' + phi on internal pressure cells, p' = f.pp).  The step itself folds this into
// the next momentum; this kernel materialises the state on request.  mode bit 0: the state goes to f.u, f.v, f.w, f.p; bit 1: it is written
// back over the predictor and the pressure it was computed from (f.us, f.pp: each point
// reads only its own), which makes it the start of the next substep once the caller
// zeroes phi and Pi.
// ---------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_correct(GridParams g, Fields<T> f, IbmLists L, int mode, double ck_dt,
                                                const double* __restrict__ pi) {
  const int i = blockIdx.x * BX + threadIdx.x;
  const int k = blockIdx.y * BZ + threadIdx.y;
  const int j = blockIdx.z;
  if (i >= g.nx || k >= g.nz) return;
  const int nx = g.nx, nz = g.nz;
  const int im = wrap_m(i, nx), km = wrap_m(k, nz);
  const int c = (j * nz + k) * nx + i;
  const int ds = (j > 0) ? nx * nz : 0;      // v on face 0 is never internal
  const Corrected<T> r = corrected_point<T>(g, f, L.wallv, f.tag[c], j, c, c - i + im, c - ds,
                                            c + (km - k) * nx, ck_dt, pi[0]);
  if (mode & 1) {
    f.u[c] = r.u;
    f.v[c] = r.v;
    f.w[c] = r.w;
    f.p[c] = r.p;
  }
  if (mode & 2) {
    f.us[c] = r.u;
    f.vs[c] = r.v;
    f.ws[c] = r.w;
    f.pp[c] = r.p;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_copy(const T* __restrict__ src, T* __restrict__ dst, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

// Streaming copy of n 16-byte vectors (the practical HBM ceiling of a kernel that reads and
// writes each byte once): one vector per thread, one block per 256 vectors (on this part
// the fastest of the forms measured: 6.1 TB/s over 2 GiB, against 5.3-5.8 TB/s for
// unrolled or grid-stride forms and 4.9 TB/s for hipMemcpy).
__global__ __launch_bounds__(256) void k_stream_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                      int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) dst[e] = src[e];
}

// Streams nsrc arrays into ndst arrays (each output the element-wise FP64 sum of the
// inputs), 16-byte vectors, one vector of every array per thread: the practical HBM
// ceiling of a kernel with the same numbers of read and write streams (a kernel of a
// step moves 5..8 read and 4..7 write streams at once, against the copy's one and one).
__global__ __launch_bounds__(256) void k_stream_mix(MixPtrs p, int nsrc, int ndst, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  double2 v[MIX_MAX];
#pragma unroll
  for (int q = 0; q < MIX_MAX; ++q)
    if (q < nsrc) v[q] = p.src[q][e];
  double2 acc = v[0];
#pragma unroll
  for (int q = 1; q < MIX_MAX; ++q)
    if (q < nsrc) {
      acc.x += v[q].x;
      acc.y += v[q].y;
    }
#pragma unroll
  for (int q = 0; q < MIX_MAX; ++q)
    if (q < ndst) p.dst[q][e] = acc;
}

}  // namespace

hipError_t launch_stream_mix(const MixPtrs& p, int nsrc, int ndst, int64_t nvec, hipStream_t st) {
  if (nvec <= 0) return hipSuccess;
  const int64_t nb = (nvec + 255) / 256;
  if (nb > 0x7fffffffll) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_stream_mix, dim3((unsigned)nb), dim3(256), 0, st, p, nsrc, ndst, nvec);
  return hipGetLastError();
}

hipError_t launch_stream_copy(const void* src, void* dst, int64_t nvec, hipStream_t st) {
  if (nvec <= 0) return hipSuccess;
  const int64_t nb = (nvec + 255) / 256;
  if (nb > 0x7fffffffll) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)nb), dim3(256), 0, st, (const uint4*)src, (uint4*)dst, nvec);
  return hipGetLastError();
}

// =======================================================================================
// Launchers
// =======================================================================================
static inline dim3 cell_grid(const GridParams& g) {
  return dim3((g.nx + BX - 1) / BX, (g.nz + BZ - 1) / BZ, g.ny1);
}

// Momentum tile variant launched for a tuning: 0 64 x 4 (automatic), 2 128 x 4, 3 64 x 8,
// 4 256 x 4, 5 128 x 8, 6 64 x 4 with two planes of loads in flight.  The two largest fit
// the LDS only in FP32 storage, and stretched grids have the 64 x 4 kernel only: those
// cases launch the 64 x 4 tile (variant 0).
static int momentum_variant(const GridParams& g, const Tuning& tu, size_t esize) {
  int t = (tu.mom_tile >= 0 && tu.mom_tile < 7) ? tu.mom_tile : 0;
  if (t == 1 || g.stretched || (esize != 4 && (t == 4 || t == 5))) t = 0;
  return t;
}
static void momentum_tile(int variant, int* tx, int* tz) {
  static const int TXS[7] = {64, 64, 128, 64, 256, 128, 64}, TZS[7] = {4, 4, 4, 8, 4, 8, 4};
  *tx = TXS[variant];
  *tz = TZS[variant];
}

// y planes per momentum block: about 2048 blocks, 4..64 planes each, unless tuned.
static int momentum_chunk(const GridParams& g, const Tuning& tu, size_t esize) {
  if (tu.mom_jc > 0) return tu.mom_jc < g.ny1 ? tu.mom_jc : g.ny1;
  int MX, MZ;
  momentum_tile(momentum_variant(g, tu, esize), &MX, &MZ);
  const long cols = (long)((g.nx + MX - 1) / MX) * ((g.nz + MZ - 1) / MZ);
  long jc = (g.ny1 * cols + 2047) / 2048;
  if (jc < 4) jc = 4;
  if (jc > 64) jc = 64;
  return (int)jc;
}

template <typename T>
hipError_t launch_momentum(const GridParams& g, const Fields<T>& f, const IbmLists& L, const StageConsts& s,
                           const double* pi_prev, double ckdt_prev, const Tuning& tu, double* qpart, int* nqpart,
                           hipStream_t st) {
  const int var = momentum_variant(g, tu, sizeof(T));
  const int jc = momentum_chunk(g, tu, sizeof(T));
  int tx, tz;
  momentum_tile(var, &tx, &tz);
  const int ntx = (g.nx + tx - 1) / tx, ntz = (g.nz + tz - 1) / tz, nty = (g.ny1 + jc - 1) / jc;
  const int nb = ntx * ntz * nty;
  const int cache = tu.mom_cache > 0 ? tu.mom_cache - 1 : 0;
  int xo = (tu.tile_order == 2 ? 0 : MOM_XCD_CONTIG) | ((cache & 1) ? MOM_NT_STORE : 0) |
           ((cache & 2) ? MOM_NT_LOAD : 0);
  if (tu.tile_order >= 3) {
    // super-tile orders (log2 of the super-tile's tiles in x and z); a grid whose tile
    // counts do not divide into whole super-tiles dealt evenly to the XCDs falls back to
    // the interleaved order
    static const int LSX[6] = {1, 2, 1, 2, 3, 3}, LSZ[6] = {1, 1, 2, 2, 1, 2};
    const int o = tu.tile_order - 3 < 6 ? tu.tile_order - 3 : 0;
    const int sx = 1 << LSX[o], sz = 1 << LSZ[o];
    xo &= ~MOM_XCD_CONTIG;
    if (ntx % sx == 0 && ntz % sz == 0 && ((ntx / sx) * (ntz / sz) * nty) % NXCD == 0)
      xo |= (LSX[o] << MOM_SUPER_SHIFT) | (LSZ[o] << (MOM_SUPER_SHIFT + 2));
  }
#define IBM_LAUNCH_MOM(SYV, TXV, TZV)                                                                   \
  hipLaunchKernelGGL((k_momentum<T, SYV, TXV, TZV>), dim3(nb), dim3(TXV, TZV), 0, st, g, f, L, s, jc, ntx, ntz, xo, \
                     pi_prev, ckdt_prev, qpart)
  if (g.stretched) {
    IBM_LAUNCH_MOM(true, 64, 4);
  } else if (var == 6) {
    hipLaunchKernelGGL((k_momentum<T, false, 64, 4, 2>), dim3(nb), dim3(64, 4), 0, st, g, f, L, s, jc, ntx, ntz, xo,
                       pi_prev, ckdt_prev, qpart);
  } else if (var == 2) {
    IBM_LAUNCH_MOM(false, 128, 4);
  } else if (var == 3) {
    IBM_LAUNCH_MOM(false, 64, 8);
  } else if (var == 4 || var == 5) {
    if constexpr (sizeof(T) == 4) {   // (momentum_variant gives these in FP32 only)
      if (var == 4) IBM_LAUNCH_MOM(false, 256, 4);
      else IBM_LAUNCH_MOM(false, 128, 8);
    }
  } else {
    IBM_LAUNCH_MOM(false, 64, 4);
  }
#undef IBM_LAUNCH_MOM
  *nqpart = nb;
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cfr_pi(const Fields<T>& f, const IbmLists& L, int stage, double ck_dt, const double* qpart, int nq,
                         double scale, int forcing, double q_target_or_pi, const double* S3, double* pi_out,
                         double* pi_hist, hipStream_t st) {
  const int nb = L.n_cover > 0 ? (L.n_cover + 255) / 256 : 1;
  hipLaunchKernelGGL(k_cfr_pi<T>, dim3(nb), dim3(256), 0, st, f, L, stage, ck_dt, qpart, nq, scale, forcing,
                     q_target_or_pi, S3, pi_out, pi_hist);
  return hipGetLastError();
}

// Row geometry of the x transforms (div_fftx, ifftx): 2^ll lanes per row, the fewest (a
// power of two from 4 to a wavefront) that keep every stage at one butterfly per lane;
// 256 threads per block, so 256 >> ll rows per block.
struct XfftShape {
  int ll, rows, mb;
  size_t lds;
};
template <typename T>
static XfftShape xfft_shape(const GridParams& g, const FFTPlan& px) {
  int l = IBM_WAVE;
  while (l > 4 && fft_max_bfly(px, l / 2) == 1) l >>= 1;
  XfftShape s;
  s.ll = __builtin_ctz((unsigned)l);
  s.rows = 256 / l;
  s.mb = fft_max_bfly(px, l);
  s.lds = (size_t)(s.rows + 1) * g.nhalf * sizeof(cplx<T>);   // rows plus the twiddle table
  return s;
}

template <typename T>
hipError_t launch_div_fftx(const GridParams& g, const Fields<T>& f, const IbmLists& L, int stage,
                           const FFTPlan& px, const double2* rtw, double ck_dt, const double* pi, const T* rhs_in,
                           hipStream_t st) {
  const XfftShape x = xfft_shape<T>(g, px);
  const int mb = x.mb, ll = x.ll;
  const size_t lds = x.lds;
  const void* k = mb == 1 ? (const void*)k_div_fftx<T, 1> : (mb == 2 ? (const void*)k_div_fftx<T, 2> : (const void*)k_div_fftx<T, 4>);
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const dim3 grid((g.nrows + x.rows - 1) / x.rows), blk(256);
  if (mb == 1) hipLaunchKernelGGL((k_div_fftx<T, 1>), grid, blk, lds, st, g, f, L, stage, px, rtw, ck_dt, pi, rhs_in, ll);
  else if (mb == 2) hipLaunchKernelGGL((k_div_fftx<T, 2>), grid, blk, lds, st, g, f, L, stage, px, rtw, ck_dt, pi, rhs_in, ll);
  else hipLaunchKernelGGL((k_div_fftx<T, 4>), grid, blk, lds, st, g, f, L, stage, px, rtw, ck_dt, pi, rhs_in, ll);
  return hipGetLastError();
}

// Threads of a z-FFT block of width W (x modes): 256, or 512 when 256 would leave
// more than two butterflies per thread in the largest stage.
static int fftz_threads(const FFTPlan& pz, int W) {
  int nbmax = 1;
  for (int s = 0; s < pz.nst; ++s) nbmax = nbmax > pz.n / pz.radix[s] ? nbmax : pz.n / pz.radix[s];
  return (W <= 256 && (nbmax + 256 / W - 1) / (256 / W) > 2 && W <= 512) ? 512 : 256;
}

// A z-FFT width W is valid when the block's threads give each column enough lanes for the
// in-place stages (<= 4 butterflies per thread) and the tile plus twiddles fit the
// 160 KiB of LDS a gfx950 workgroup may hold.
template <typename T>
static bool fftz_width_ok(const GridParams& g, const FFTPlan& pz, int W) {
  if (W < 1 || W > 256 || 256 % W) return false;
  const int nt = fftz_threads(pz, W);
  int nbmax = 1;
  for (int s = 0; s < pz.nst; ++s) nbmax = nbmax > pz.n / pz.radix[s] ? nbmax : pz.n / pz.radix[s];
  if ((nbmax + nt / W - 1) / (nt / W) > 4) return false;
  return ((size_t)W + 1) * g.nz * sizeof(cplx<T>) <= 163840;
}

template <typename T>
int fftz_widths(const GridParams& g, const FFTPlan& pz, int* out, int max) {
  int n = 0;
  for (int W = 1; W <= 64 && n < max; W <<= 1)
    if (fftz_width_ok<T>(g, pz, W)) out[n++] = W;
  return n;
}

// Default: 128-byte rows (8 FP64 / 16 FP32 complex values) or the widest valid below.
template <typename T>
static int fftz_width(const GridParams& g, const FFTPlan& pz, const Tuning& tu) {
  if (tu.fftz_w > 0 && fftz_width_ok<T>(g, pz, tu.fftz_w)) return tu.fftz_w;
  int W = (int)(128 / sizeof(cplx<T>));
  while (W > 1 && !fftz_width_ok<T>(g, pz, W)) W >>= 1;
  return W;
}

template <typename T, int MB, int RP>
static hipError_t launch_fftz_v(const GridParams& g, cplx<T>* spec, const FFTPlan& pz, int sign, int W, int NJ,
                                int nt, size_t lds, hipStream_t st) {
  const void* kfn = (const void*)k_fftz<T, MB, RP>;
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_fftz<T, MB, RP>), dim3(fftz_blocks(g.mh, g.ny1, W, NJ)), dim3(nt), lds, st, g, spec, pz,
                     sign, W, NJ);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fftz(const GridParams& g, cplx<T>* spec, const FFTPlan& pz, int sign, const Tuning& tu,
                       hipStream_t st) {
  const int W = fftz_width<T>(g, pz, tu);
  const int nt = fftz_threads(pz, W);
  const size_t lds = ((size_t)W + 1) * g.nz * sizeof(cplx<T>);
  const int mb = fft_max_bfly(pz, nt / W);
  // planes per block: two, with the next plane's columns held in registers, when a
  // thread's share of a column (ceil(nz / lanes)) fits 4 or 8 registers
  const int per = (g.nz + nt / W - 1) / (nt / W);
  const int rp = per <= 4 ? 4 : (per <= 8 ? 8 : 0);
  const int nj = rp ? 2 : 1;
  if (mb == 1) {
    if (rp == 4) return launch_fftz_v<T, 1, 4>(g, spec, pz, sign, W, nj, nt, lds, st);
    if (rp == 8) return launch_fftz_v<T, 1, 8>(g, spec, pz, sign, W, nj, nt, lds, st);
    return launch_fftz_v<T, 1, 0>(g, spec, pz, sign, W, nj, nt, lds, st);
  }
  if (mb == 2) {
    if (rp == 4) return launch_fftz_v<T, 2, 4>(g, spec, pz, sign, W, nj, nt, lds, st);
    if (rp == 8) return launch_fftz_v<T, 2, 8>(g, spec, pz, sign, W, nj, nt, lds, st);
    return launch_fftz_v<T, 2, 0>(g, spec, pz, sign, W, nj, nt, lds, st);
  }
  if (rp == 4) return launch_fftz_v<T, 4, 4>(g, spec, pz, sign, W, nj, nt, lds, st);
  if (rp == 8) return launch_fftz_v<T, 4, 8>(g, spec, pz, sign, W, nj, nt, lds, st);
  return launch_fftz_v<T, 4, 0>(g, spec, pz, sign, W, nj, nt, lds, st);
}

// Modes per tridiagonal block with P threads per mode in at most tb threads: tb / P, or the
// largest power of two below it when that is at least 8 (whole 128-byte lines of every row
// in FP64, half lines in FP32; a run of W modes that is not a power of two starts and ends
// inside lines, and its segment groups straddle the wavefronts).
static int tri_width(int P, int tb) {
  int w2 = 1;
  while (2 * w2 * P <= tb) w2 *= 2;
  return w2 >= 8 ? w2 : tb / P;
}

template <typename T>
hipError_t launch_tri(const GridParams& g, cplx<T>* spec, const double* kx2, const double* kz2, double* mean_out,
                      const Tuning& tu, hipStream_t st) {
  const int n = g.ny1;
  const int L = (tu.tri_rows == 4) ? 4 : 8;  // rows per thread
  int P = (n + L - 1) / L;                   // segments of at most L rows ...
  if (P > n / 2) P = n / 2 > 0 ? n / 2 : 1;  // ... and at least 2
  if (P > 256) P = 256;
  // 128-thread blocks while their modes still fill whole 128-byte lines of every row read:
  // twice the blocks of 256 threads spread more evenly over the compute units
  const int TBM = (128 / P) * (int)sizeof(cplx<T>) >= 128 ? 128 : 256;
  const int W = tri_width(P, TBM);        // modes per block
  const int TB = W * P;
  const size_t lds = (size_t)(4 * tri_rs(W) * 2 * P + 2 * P) * sizeof(double);
  const int gather = tri_gather(g);
  const dim3 grid(tri_blocks(g, W, gather));
  const bool l4 = L == 4 && (n + P - 1) / P <= 4;
  if (g.stretched) {
    if (l4) hipLaunchKernelGGL((k_tri<T, 4, true>), grid, dim3(TB), lds, st, g, spec, kx2, kz2, P, W, mean_out,
                                          gather);
    else hipLaunchKernelGGL((k_tri<T, 8, true>), grid, dim3(TB), lds, st, g, spec, kx2, kz2, P, W, mean_out,
                                          gather);
  } else {
    if (l4) hipLaunchKernelGGL((k_tri<T, 4, false>), grid, dim3(TB), lds, st, g, spec, kx2, kz2, P, W, mean_out,
                                          gather);
    else hipLaunchKernelGGL((k_tri<T, 8, false>), grid, dim3(TB), lds, st, g, spec, kx2, kz2, P, W, mean_out,
                                          gather);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ifftx(const GridParams& g, const cplx<T>* spec, T* out, const FFTPlan& px, const double2* rtw,
                        hipStream_t st) {
  const XfftShape x = xfft_shape<T>(g, px);
  const int mb = x.mb, ll = x.ll;
  const size_t lds = x.lds;
  const void* k = mb == 1 ? (const void*)k_ifftx<T, 1> : (mb == 2 ? (const void*)k_ifftx<T, 2> : (const void*)k_ifftx<T, 4>);
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const dim3 grid((g.nrows + x.rows - 1) / x.rows);
  if (mb == 1) hipLaunchKernelGGL((k_ifftx<T, 1>), grid, dim3(256), lds, st, g, spec, out, px, rtw, ll);
  else if (mb == 2) hipLaunchKernelGGL((k_ifftx<T, 2>), grid, dim3(256), lds, st, g, spec, out, px, rtw, ll);
  else hipLaunchKernelGGL((k_ifftx<T, 4>), grid, dim3(256), lds, st, g, spec, out, px, rtw, ll);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_correct(const GridParams& g, const Fields<T>& f, const IbmLists& L, int mode, double ck_dt,
                          const double* pi, hipStream_t st) {
  hipLaunchKernelGGL(k_correct<T>, cell_grid(g), dim3(BX, BZ), 0, st, g, f, L, mode, ck_dt, pi);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_copy(const T* src, T* dst, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t nb = (n + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_copy<T>, dim3((unsigned)nb), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

// =======================================================================================
// Batched launches: the step kernels of many independent grids in one launch each.  The
// plan_* functions fill one grid's arguments exactly as the single-grid launchers choose
// them and return its number of blocks; the batched launch takes the per-grid arguments
// and the block offsets from device memory and uses the largest template variant and
// LDS size any grid needs (the kernels read the per-grid sizes at run time).
// =======================================================================================
template <typename T>
int plan_momentum(const GridParams& g, const Fields<T>& f, const IbmLists& L, const StageConsts& s,
                  const double* pi_prev, double ckdt_prev, const Tuning& tu0, double* qpart, MomArgs<T>* a) {
  Tuning tu = tu0;
  tu.mom_tile = 0;   // batched launches use the default tile
  const int jc = momentum_chunk(g, tu, sizeof(T));
  const int ntx = (g.nx + MX - 1) / MX, ntz = (g.nz + MZ - 1) / MZ, nty = (g.ny1 + jc - 1) / jc;
  const int nb = ntx * ntz * nty;
  *a = MomArgs<T>{g, f, L, s, jc, ntx, ntz, 0, pi_prev, ckdt_prev, qpart, nb};
  return nb;
}

template <typename T>
int plan_cfr_pi(const Fields<T>& f, const IbmLists& L, int stage, double ck_dt, const double* qpart, int nq,
                double scale, int forcing, double q_target_or_pi, const double* S3, double* pi_out, double* pi_hist,
                CfrArgs<T>* a) {
  const int nb = L.n_cover > 0 ? (L.n_cover + 255) / 256 : 1;
  *a = CfrArgs<T>{f, L, stage, ck_dt, qpart, nq, scale, forcing, q_target_or_pi, S3, pi_out, pi_hist, nb};
  return nb;
}

template <typename T>
int plan_div_fftx(const GridParams& g, const Fields<T>& f, const IbmLists& L, int stage, const FFTPlan& px,
                  const double2* rtw, double ck_dt, const double* pi, DivArgs<T>* a, int* mb, size_t* lds) {
  const XfftShape x = xfft_shape<T>(g, px);
  const int nb = (g.nrows + x.rows - 1) / x.rows;
  *a = DivArgs<T>{g, f, L, stage, px, rtw, ck_dt, pi, (const T*)nullptr, x.ll, nb};
  *mb = x.mb;
  *lds = x.lds;
  return nb;
}

template <typename T>
int plan_fftz(const GridParams& g, cplx<T>* spec, const FFTPlan& pz, int sign, const Tuning& tu, FftzArgs<T>* a,
              int* mb, size_t* lds, int* threads) {
  const int W = fftz_width<T>(g, pz, tu);
  const int nt = fftz_threads(pz, W);
  const int nb = fftz_blocks(g.mh, g.ny1, W, 1);
  *a = FftzArgs<T>{g, spec, pz, sign, W, nb, 1};
  *mb = fft_max_bfly(pz, nt / W);
  *lds = ((size_t)W + 1) * g.nz * sizeof(cplx<T>);
  *threads = nt;
  return nb;
}

template <typename T>
int plan_tri(const GridParams& g, cplx<T>* spec, const double* kx2, const double* kz2, double* mean_out,
             const Tuning& tu, TriArgs<T>* a, int* lm, size_t* lds) {
  const int n = g.ny1;
  const int L = (tu.tri_rows == 4) ? 4 : 8;
  int P = (n + L - 1) / L;
  if (P > n / 2) P = n / 2 > 0 ? n / 2 : 1;
  if (P > 256) P = 256;
  const int W = 256 / P;   // (the launch's 256 threads: a power-of-two W would leave some idle)
  const int gather = tri_gather(g);
  const int nb = tri_blocks(g, W, gather);
  *a = TriArgs<T>{g, spec, kx2, kz2, P, W, mean_out, nb, gather};
  *lm = (L == 4 && (n + P - 1) / P <= 4) ? 4 : 8;
  *lds = (size_t)(4 * tri_rs(W) * 2 * P + 2 * P) * sizeof(double);
  return nb;
}

template <typename T>
int plan_ifftx(const GridParams& g, const cplx<T>* spec, T* out, const FFTPlan& px, const double2* rtw,
               IfftxArgs<T>* a, int* mb, size_t* lds) {
  const XfftShape x = xfft_shape<T>(g, px);
  const int nb = (g.nrows + x.rows - 1) / x.rows;
  *a = IfftxArgs<T>{g, spec, out, px, rtw, x.ll, nb};
  *mb = x.mb;
  *lds = x.lds;
  return nb;
}

// Dynamic LDS above 64 KiB has to be allowed per kernel.
static hipError_t allow_lds(const void* kfn, size_t lds) {
  if (lds <= 65536) return hipSuccess;
  return hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <typename T>
hipError_t launch_momentum_b(const MomArgs<T>* args, const int* boff, int ninst, int ntot, bool stretched,
                             hipStream_t st) {
  if (stretched)
    hipLaunchKernelGGL((k_momentum_b<T, true>), dim3(ntot), dim3(MX, MZ), 0, st, args, boff, ninst);
  else
    hipLaunchKernelGGL((k_momentum_b<T, false>), dim3(ntot), dim3(MX, MZ), 0, st, args, boff, ninst);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cfr_pi_b(const CfrArgs<T>* args, const int* boff, int ninst, int ntot, hipStream_t st) {
  hipLaunchKernelGGL(k_cfr_pi_b<T>, dim3(ntot), dim3(256), 0, st, args, boff, ninst);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_div_fftx_b(const DivArgs<T>* args, const int* boff, int ninst, int ntot, int mb, size_t lds,
                             hipStream_t st) {
  const void* k = mb == 1 ? (const void*)k_div_fftx_b<T, 1> : (mb == 2 ? (const void*)k_div_fftx_b<T, 2> : (const void*)k_div_fftx_b<T, 4>);
  hipError_t e = allow_lds(k, lds);
  if (e != hipSuccess) return e;
  if (mb == 1) hipLaunchKernelGGL((k_div_fftx_b<T, 1>), dim3(ntot), dim3(256), lds, st, args, boff, ninst);
  else if (mb == 2) hipLaunchKernelGGL((k_div_fftx_b<T, 2>), dim3(ntot), dim3(256), lds, st, args, boff, ninst);
  else hipLaunchKernelGGL((k_div_fftx_b<T, 4>), dim3(ntot), dim3(256), lds, st, args, boff, ninst);
  return hipGetLastError();
}

template <typename T, int MB, int RP>
static hipError_t launch_fftz_bv(const FftzArgs<T>* args, const int* boff, int ninst, int ntot, size_t lds,
                                 int threads, hipStream_t st) {
  hipError_t e = allow_lds((const void*)k_fftz_b<T, MB, RP>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_fftz_b<T, MB, RP>), dim3(ntot), dim3(threads), lds, st, args, boff, ninst);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fftz_b(const FftzArgs<T>* args, const int* boff, int ninst, int ntot, int mb, int rp, size_t lds,
                         int threads, hipStream_t st) {
  if (rp != 0 && rp != 4 && rp != 8) return hipErrorInvalidValue;
  if (mb == 1) {
    if (rp == 4) return launch_fftz_bv<T, 1, 4>(args, boff, ninst, ntot, lds, threads, st);
    if (rp == 8) return launch_fftz_bv<T, 1, 8>(args, boff, ninst, ntot, lds, threads, st);
    return launch_fftz_bv<T, 1, 0>(args, boff, ninst, ntot, lds, threads, st);
  }
  if (mb == 2) {
    if (rp == 4) return launch_fftz_bv<T, 2, 4>(args, boff, ninst, ntot, lds, threads, st);
    if (rp == 8) return launch_fftz_bv<T, 2, 8>(args, boff, ninst, ntot, lds, threads, st);
    return launch_fftz_bv<T, 2, 0>(args, boff, ninst, ntot, lds, threads, st);
  }
  if (rp == 4) return launch_fftz_bv<T, 4, 4>(args, boff, ninst, ntot, lds, threads, st);
  if (rp == 8) return launch_fftz_bv<T, 4, 8>(args, boff, ninst, ntot, lds, threads, st);
  return launch_fftz_bv<T, 4, 0>(args, boff, ninst, ntot, lds, threads, st);
}

template <typename T>
hipError_t launch_tri_b(const TriArgs<T>* args, const int* boff, int ninst, int ntot, int lm, size_t lds,
                        bool stretched, hipStream_t st) {
  const void* k = stretched ? (lm == 4 ? (const void*)k_tri_b<T, 4, true> : (const void*)k_tri_b<T, 8, true>)
                            : (lm == 4 ? (const void*)k_tri_b<T, 4, false> : (const void*)k_tri_b<T, 8, false>);
  hipError_t e = allow_lds(k, lds);
  if (e != hipSuccess) return e;
  if (stretched) {
    if (lm == 4) hipLaunchKernelGGL((k_tri_b<T, 4, true>), dim3(ntot), dim3(256), lds, st, args, boff, ninst);
    else hipLaunchKernelGGL((k_tri_b<T, 8, true>), dim3(ntot), dim3(256), lds, st, args, boff, ninst);
  } else {
    if (lm == 4) hipLaunchKernelGGL((k_tri_b<T, 4, false>), dim3(ntot), dim3(256), lds, st, args, boff, ninst);
    else hipLaunchKernelGGL((k_tri_b<T, 8, false>), dim3(ntot), dim3(256), lds, st, args, boff, ninst);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ifftx_b(const IfftxArgs<T>* args, const int* boff, int ninst, int ntot, int mb, size_t lds,
                          hipStream_t st) {
  const void* k = mb == 1 ? (const void*)k_ifftx_b<T, 1> : (mb == 2 ? (const void*)k_ifftx_b<T, 2> : (const void*)k_ifftx_b<T, 4>);
  hipError_t e = allow_lds(k, lds);
  if (e != hipSuccess) return e;
  if (mb == 1) hipLaunchKernelGGL((k_ifftx_b<T, 1>), dim3(ntot), dim3(256), lds, st, args, boff, ninst);
  else if (mb == 2) hipLaunchKernelGGL((k_ifftx_b<T, 2>), dim3(ntot), dim3(256), lds, st, args, boff, ninst);
  else hipLaunchKernelGGL((k_ifftx_b<T, 4>), dim3(ntot), dim3(256), lds, st, args, boff, ninst);
  return hipGetLastError();
}

#define IBM_BATCH_INST(T)                                                                                        \
  template int plan_momentum<T>(const GridParams&, const Fields<T>&, const IbmLists&, const StageConsts&,       \
                                const double*, double, const Tuning&, double*, MomArgs<T>*);                    \
  template int plan_cfr_pi<T>(const Fields<T>&, const IbmLists&, int, double, const double*, int, double, int,  \
                              double, const double*, double*, double*, CfrArgs<T>*);                            \
  template int plan_div_fftx<T>(const GridParams&, const Fields<T>&, const IbmLists&, int, const FFTPlan&,      \
                                const double2*, double, const double*, DivArgs<T>*, int*, size_t*);             \
  template int plan_fftz<T>(const GridParams&, cplx<T>*, const FFTPlan&, int, const Tuning&, FftzArgs<T>*,      \
                            int*, size_t*, int*);                                                               \
  template int plan_tri<T>(const GridParams&, cplx<T>*, const double*, const double*, double*, const Tuning&,   \
                           TriArgs<T>*, int*, size_t*);                                                         \
  template int plan_ifftx<T>(const GridParams&, const cplx<T>*, T*, const FFTPlan&, const double2*,             \
                             IfftxArgs<T>*, int*, size_t*);                                                     \
  template hipError_t launch_momentum_b<T>(const MomArgs<T>*, const int*, int, int, bool, hipStream_t);               \
  template hipError_t launch_cfr_pi_b<T>(const CfrArgs<T>*, const int*, int, int, hipStream_t);                 \
  template hipError_t launch_div_fftx_b<T>(const DivArgs<T>*, const int*, int, int, int, size_t, hipStream_t);  \
  template hipError_t launch_fftz_b<T>(const FftzArgs<T>*, const int*, int, int, int, int, size_t, int,         \
                                       hipStream_t);                                                            \
  template hipError_t launch_tri_b<T>(const TriArgs<T>*, const int*, int, int, int, size_t, bool, hipStream_t);       \
  template hipError_t launch_ifftx_b<T>(const IfftxArgs<T>*, const int*, int, int, int, size_t, hipStream_t);

IBM_BATCH_INST(double)
IBM_BATCH_INST(float)

#define IBM_INST(T)                                                                                              \
  template hipError_t launch_momentum<T>(const GridParams&, const Fields<T>&, const IbmLists&,                  \
                                         const StageConsts&, const double*, double, const Tuning&, double*,      \
                                         int*, hipStream_t);                                                     \
  template hipError_t launch_cfr_pi<T>(const Fields<T>&, const IbmLists&, int, double, const double*, int,      \
                                       double, int, double, const double*, double*, double*, hipStream_t);       \
  template hipError_t launch_div_fftx<T>(const GridParams&, const Fields<T>&, const IbmLists&, int,             \
                                         const FFTPlan&, const double2*, double, const double*, const T*,        \
                                         hipStream_t);                                                           \
  template hipError_t launch_fftz<T>(const GridParams&, cplx<T>*, const FFTPlan&, int, const Tuning&,           \
                                     hipStream_t);                                                               \
  template int fftz_widths<T>(const GridParams&, const FFTPlan&, int*, int);                                    \
  template hipError_t launch_tri<T>(const GridParams&, cplx<T>*, const double*, const double*, double*,         \
                                    const Tuning&, hipStream_t);                                                 \
  template hipError_t launch_ifftx<T>(const GridParams&, const cplx<T>*, T*, const FFTPlan&, const double2*,    \
                                      hipStream_t);                                                              \
  template hipError_t launch_correct<T>(const GridParams&, const Fields<T>&, const IbmLists&, int, double,      \
                                        const double*, hipStream_t);                                             \
  template hipError_t launch_copy<T>(const T*, T*, int64_t, hipStream_t);

IBM_INST(double)
IBM_INST(float)
