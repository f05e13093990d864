// Single-pass step: one HBM read and one HBM write of every population.
//
// The Shan-Chen force at x needs psi of the *same* time level at the 18
// neighbours of x, and psi there needs those neighbours' populations.  A
// workgroup therefore owns a column of TX x TY nodes and marches through a
// chunk of z-planes, keeping psi of four consecutive planes of its tile plus
// a one-node halo ring in an LDS ring buffer.  The tile's own populations
// are read from HBM once and stay in registers until their plane is
// collided; the halo's populations belong to neighbouring columns that are
// marched at the same time, so re-reading them mostly hits the caches.  Each
// chunk also reads the plane before and the plane after it.  (This
// describes k_fused, the float32 / float16 kernel; the float64 kernel
// k_fused_pair further down is described there.)
//
// Software pipeline of depth D >= 2 (one barrier per plane): iteration z
// issues the loads of plane z + D, collides plane z (psi of z - 1, z, z + 1
// are already in LDS) and pushes its post-collision populations, then turns
// the plane z + D loads into psi.  The loads are in flight during D
// collisions' worth of work, and since they are issued before that plane's
// stores, waiting for them never waits for the stores.  Interior populations
// of planes z .. z + D - 1 stay in registers.
//
// Lane layout: each wave carries one component for one row of TX = 64 nodes
// or two rows of TX = 32, so every population plane it touches has a
// wave-uniform base address.  The other component's
// density and momentum at the same node, needed for the common velocity,
// come from an LDS exchange written one iteration ahead.
//
// Streaming is push: f*_i(x) goes to x + c_i in the other grid, or back into
// (x, opp(i)) when x + c_i is solid.  Both grids hold pre-collision
// populations in the library's structure-of-arrays layout.
//
// Workgroups are numbered so that the ones the hardware sends to the same
// XCD (workgroup id modulo 8) take a contiguous run of tiles of one z-chunk
// (see fused_work_item): neighbouring columns then share that XCD's L2 for
// their halo reads.
#pragma once

#include "lb_kernels.h"

namespace lbd {

constexpr int kFusedTX = 32;
constexpr int kXCDs = 8;
// collision model of the component-pair kernel
constexpr int kModelSC = 0;  // Shan-Chen pseudopotential force, velocity shift
constexpr int kModelCG = 1;  // colour gradient: BGK + perturbation + recolouring

// Workgroup barrier that orders LDS accesses only.  The waves of a fused
// workgroup exchange data through LDS alone (the kernels never read what
// they write to global memory), so global stores -- and register loads
// issued ahead -- may stay in flight across it.  __syncthreads() would wait
// for every outstanding vector memory operation of the wave at each barrier.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

struct FusedTiling {
  int tiles_x, tiles_y;  // tile counts along x and y
  int chunk;             // planes per z-chunk
  int chunks;            // number of z-chunks
  int total;             // tiles_x * tiles_y * chunks
  int per_round;         // workgroups resident at once (compute units x workgroups per unit), a multiple of 8
};

// Workgroup id -> work item.  Workgroups are dispatched in id order, round
// after round of `per_round`, and id modulo 8 picks the XCD.  Within each
// round the XCD-contiguous numbering above applies, so that the columns
// resident at one time form one compact block of consecutive tiles (their
// halo rows then come from columns being marched at the same time, and
// x-neighbours share an XCD's L2).
__device__ __forceinline__ int fused_work_item(int b, int total, int per_round) {
  const int base = (b / per_round) * per_round;
  const int n = min(per_round, total - base);
  const int bb = b - base;
  const int q = n / kXCDs, r = n % kXCDs;
  const int j = bb % kXCDs, s = bb / kXCDs;
  return base + j * q + (j < r ? j : r) + s;
}


// State between the structure-of-arrays layout (plane ki at ki * Npad, node
// n = x + nx (y + ny z)) and the tile-major one; to_tiled selects the
// direction.  One work-item per node, 38 values each.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_relayout(const T* __restrict__ src, T* __restrict__ dst, Geometry g,
                                                     int to_tiled) {
  const long long n = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (n >= g.N) return;
  const int x = (int)(n % g.nx), y = (int)((n / g.nx) % g.ny), z = (int)(n / ((long long)g.nx * g.ny));
  const long long t = tile_major_index(0, x, y, z, g);
#pragma unroll
  for (int ki = 0; ki < 2 * Q; ++ki) {
    const long long s = (long long)ki * g.Npad + n, d = t + (long long)ki * kTileNodes;
    if (to_tiled) dst[d] = src[s];
    else dst[s] = src[d];
  }
}

// RECORD: also write the moment record of the pre-collision state (rho_A,
// rho_B, m_A, m_B, psi_A, psi_B as [10][N], zero at solid nodes) that the
// adjoint step consumes.
//
// TX = 32: each wave carries two rows of 32 nodes; TX = 64: one row of 64
// (whole 128-byte lines of float16 rows, fewer partly written lines at the
// tile's x edges).  A workgroup has 2 TY / (64 / TX) waves.
//
// TILED: the populations are in the tile-major layout (TX = 64); only the
// addressing differs.
//
// LEAD: the loads of a plane are issued LEAD iterations before its psi is
// published.  LEAD = 1: plane z + D is loaded at the start of the iteration
// that collides plane z and published at its end, so the loads have one
// collision to land.  LEAD = 2: plane z + D + 1 is loaded instead and
// published one iteration later, two collisions after its loads were issued,
// at the cost of one more plane of populations (and halo) in registers.
template <int ST, bool SOLID, int TY, int D, bool RECORD, int TX = kFusedTX, bool TILED = false, int LEAD = 1>
__global__ void __launch_bounds__(128 * TY * TX / 64) k_fused(const store_t<ST>* __restrict__ fin,
                                                              store_t<ST>* __restrict__ fout,
                                                              const uint8_t* __restrict__ mask, Geometry g,
                                                              StepCoeffs c, FusedTiling t,
                                                              real_t<ST>* __restrict__ rec) {
  using real = real_t<ST>;
  using store = store_t<ST>;
  constexpr int RPW = 64 / TX;             // rows per wave
  constexpr int RX = TX + 2, RY = TY + 2;  // ring plane incl. halo
  constexpr int NS = D + 2;                // ring slots: planes z - 1 .. z + D
  constexpr int NX = D + 1;                // exchange slots: planes z .. z + D
  constexpr bool CORNERS_IN_ROWS = RX <= 64;  // else the four corners go with the side columns
  static_assert(D >= 2, "psi of plane z + 1 must be ready before plane z is collided");
  static_assert(LEAD == 1 || LEAD == 2, "loads one or two iterations ahead of their publication");
  static_assert(sizeof(real) == 4, "float arithmetic only; float64 storage runs k_fused_pair");
  static_assert(TX == 32 || TX == 64, "a wave covers two rows of 32 or one row of 64");
  static_assert(TY % RPW == 0 && TY / RPW >= 3, "three waves per component carry the halo");
  static_assert(2 * TY + (CORNERS_IN_ROWS ? 0 : 4) <= 64, "one wave carries the side columns");
  static_assert(!TILED || (TX == kTileX && TY % kTileY == 0), "tile-major rows are 64 nodes, tiles 4 rows");
  __shared__ real ring[NS][2][RY][RX];
  __shared__ real xch[NX][2][4][TY][TX];  // [plane slot][component][rho, mx, my, mz][y][x]
  __shared__ uint8_t ring_solid[SOLID ? NS : 1][SOLID ? RY : 1][SOLID ? RX : 1];

  const int w = fused_work_item(blockIdx.x, t.total, t.per_round);
  const int chunk = w / (t.tiles_x * t.tiles_y);
  const int tile = w - chunk * (t.tiles_x * t.tiles_y);
  const int ty0 = (tile / t.tiles_x) * TY, tx0 = (tile % t.tiles_x) * TX;
  const int z0 = chunk * t.chunk;
  const int zlen = min(t.chunk, g.nz - z0);

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int k = __builtin_amdgcn_readfirstlane(wave & 1);    // component of this wave
  const int rp = __builtin_amdgcn_readfirstlane(wave >> 1);  // row group of this wave
  const int lx = lane % TX, ly = RPW * rp + lane / TX;
  // interior node of this lane, wrapped into the box (lanes past the box edge
  // read the wrapped node so that every ring slot holds the right psi)
  const int gx = (tx0 + lx) % g.nx, gy = (ty0 + ly) % g.ny;
  const bool active = (tx0 + lx) < g.nx && (ty0 + ly) < g.ny;
  const uint32_t row = (uint32_t)gx + (uint32_t)g.nx * (uint32_t)gy;
  const uint32_t plane_n = (uint32_t)g.nx * (uint32_t)g.ny;

  // halo node of this lane: row group 0 -> row above, 1 -> row below,
  // 2 -> left and right columns (and the corners when a row has more than
  // 64 ring nodes), others none
  bool has_halo = false;
  int hx = 0, hy = 0;
  constexpr int x_lo = CORNERS_IN_ROWS ? -1 : 0, nrow = CORNERS_IN_ROWS ? RX : TX;
  if (rp == 0 && lane < nrow) { has_halo = true; hx = lane + x_lo; hy = -1; }
  if (rp == 1 && lane < nrow) { has_halo = true; hx = lane + x_lo; hy = TY; }
  if (rp == 2 && lane < 2 * TY) { has_halo = true; hx = lane < TY ? -1 : TX; hy = lane < TY ? lane : lane - TY; }
  if (!CORNERS_IN_ROWS && rp == 2 && lane >= 2 * TY && lane < 2 * TY + 4) {
    const int cn = lane - 2 * TY;
    has_halo = true;
    hx = (cn & 1) ? TX : -1;
    hy = (cn & 2) ? TY : -1;
  }
  const int hgx = ((tx0 + hx) % g.nx + g.nx) % g.nx;
  const int hgy = ((ty0 + hy) % g.ny + g.ny) % g.ny;
  const uint32_t hrow = (uint32_t)hgx + (uint32_t)g.nx * (uint32_t)hgy;

  // Plane bases are wave-uniform (scalar registers); per-lane offsets are
  // 32-bit byte offsets (the host only selects this kernel when
  // N * sizeof(store) < 2^32).
  const char* __restrict__ fk = reinterpret_cast<const char*>(fin + (size_t)(k * Q) * (size_t)g.Npad);
  char* __restrict__ ok = reinterpret_cast<char*>(fout + (size_t)(k * Q) * (size_t)g.Npad);
  const size_t pbytes = (size_t)g.Npad * sizeof(store);
  constexpr uint32_t ES = sizeof(store);

  auto wrapz = [&](int z) { return z < 0 ? z + g.nz : (z >= g.nz ? z - g.nz : z); };
  auto slot = [&](int z) { return (z - z0 + 1 + NS) % NS; };  // ring slot of plane z (z0-1 .. z0+zlen)
  auto xslot = [&](int z) { return (z - z0 + 1 + NX) % NX; };  // exchange slot of plane z
  // The iteration that collides plane z (reading psi of z - 1 .. z + 1 and the
  // exchange of z) writes plane z + D; with D + 2 ring slots and D + 1
  // exchange slots no write lands where another wave may still be reading.

  auto load19 = [&](uint32_t n, real (&v)[Q]) {
    const uint32_t b = n * ES;
#pragma unroll
    for (int i = 0; i < Q; ++i)
      v[i] = decode<ST>(*reinterpret_cast<const store*>(fk + (size_t)i * pbytes + b), c.shift[k][i]);
  };
  // TILED: the same from the in-plane byte offset tb of population plane 0
  // (tile-major) and the plane index z, by raw buffer loads: the z-plane's
  // block is the descriptor's range, the population row block of this
  // wave's component the scalar offset, tb the lane's offset.
  const size_t zbytes = (size_t)(2 * Q) * (size_t)plane_n * ES;  // < 2^32 (checked by the host)
  constexpr uint32_t kRowBlock = (uint32_t)kTileNodes * ES;        // bytes of one population's tile rows
  const uint32_t row_t = TILED ? (uint32_t)tile_major_index(0, gx, gy, 0, g) * ES : 0u;
  const uint32_t hrow_t = TILED ? (uint32_t)tile_major_index(0, hgx, hgy, 0, g) * ES : 0u;
  const float one = opaque_one();
  auto zplane = [&](const void* grid, int z) {
    return buffer_rsrc(reinterpret_cast<const char*>(grid) + (size_t)z * zbytes, (uint32_t)zbytes);
  };
  auto load19t = [&](uint32_t tb, int z, real (&v)[Q]) {
    const __amdgpu_buffer_rsrc_t r = zplane(fin, z);
#pragma unroll
    for (int i = 0; i < Q; ++i)
      v[i] = decode_mix<ST>(buffer_load<ST>(r, tb, (uint32_t)(k * Q + i) * kRowBlock), c.shift[k][i], one);
  };
  auto psi_from = [&](const real (&v)[Q], bool solid) -> real {
    if (SOLID && solid) return real(0);
    return pseudopotential(density<real>(v), coef_ref<real>(c));
  };
  // psi of plane z from loaded values -> ring; interior density and momentum -> exchange
  auto publish = [&](int z, const real (&v)[Q], const real (&h)[Q]) {
    const int s = slot(z), par = xslot(z);
    bool solid = false, hsolid = false;
    if constexpr (SOLID) {
      solid = mask[row + plane_n * (uint32_t)wrapz(z)] != 0;
      if (has_halo) hsolid = mask[hrow + plane_n * (uint32_t)wrapz(z)] != 0;
    }
    const real rho = density<real>(v);
    ring[s][k][ly + 1][lx + 1] = (SOLID && solid) ? real(0) : pseudopotential(rho, coef_ref<real>(c));
    xch[par][k][0][ly][lx] = rho;
    xch[par][k][1][ly][lx] = lattice_sum<0, 0, real>(v);
    xch[par][k][2][ly][lx] = lattice_sum<1, 0, real>(v);
    xch[par][k][3][ly][lx] = lattice_sum<2, 0, real>(v);
    if constexpr (SOLID) if (k == 0) ring_solid[s][ly + 1][lx + 1] = solid;
    if (has_halo) {
      ring[s][k][hy + 1][hx + 1] = psi_from(h, hsolid);
      if constexpr (SOLID) if (k == 0) ring_solid[s][hy + 1][hx + 1] = hsolid;
    }
  };

  // NB = D + LEAD population buffers rotate through the roles "plane z
  // (collided now)", "planes waiting", "plane z + D (published at the end of
  // this iteration)" and, with LEAD = 2, "plane z + D + 1 (loading)": plane
  // z0 + q lives in buf[q % NB] and its halo in hbuf[q % LEAD].  The loop
  // below is unrolled by a multiple of NB and LEAD so that the rotation is a
  // renaming, not register copies.
  constexpr int NB = D + LEAD;
  real buf[NB][Q], hbuf[LEAD][Q];
  auto load_plane = [&](int q, real (&v)[Q], real (&h)[Q]) {  // plane z0 + q
    if constexpr (TILED) {
      load19t(row_t, wrapz(z0 + q), v);
      if (has_halo) load19t(hrow_t, wrapz(z0 + q), h);
    } else {
      const uint32_t zo = plane_n * (uint32_t)wrapz(z0 + q);
      load19(row + zo, v);
      if (has_halo) load19(hrow + zo, h);
    }
  };
  // prologue: psi of planes z0 - 1 .. z0 + D - 1, populations of z0 .. z0 + D - 1
  // (and, LEAD = 2, the loads of plane z0 + D)
  load_plane(-1, buf[NB - 1], hbuf[0]);  // plane z0 - 1 is not collided here
  publish(z0 - 1, buf[NB - 1], hbuf[0]);
#pragma unroll
  for (int d = 0; d < D; ++d) {
    load_plane(d, buf[d], hbuf[d % LEAD]);
    publish(z0 + d, buf[d], hbuf[d % LEAD]);
  }
  if constexpr (LEAD == 2) load_plane(D, buf[D % NB], hbuf[D % LEAD]);
  __syncthreads();

  const real omk = coef_om<real>(c, k), omck = coef_omc<real>(c, k), tgk = coef_tg<real>(c, k);
  const real omA = coef_om<real>(c, 0), omB = coef_om<real>(c, 1);
  const int xm = gx == 0 ? g.nx - 1 : gx - 1, xp = gx == g.nx - 1 ? 0 : gx + 1;
  const int ym = gy == 0 ? g.ny - 1 : gy - 1, yp = gy == g.ny - 1 ? 0 : gy + 1;
  const uint32_t X[3] = {(uint32_t)xm, (uint32_t)gx, (uint32_t)xp};
  const uint32_t Y[3] = {(uint32_t)g.nx * ym, (uint32_t)g.nx * gy, (uint32_t)g.nx * yp};
  // TILED: in-plane byte offsets of the nine (x +- 1, y +- 1) destinations
  uint32_t T9[3][3] = {};
  if constexpr (TILED) {
    const int xs3[3] = {xm, gx, xp}, ys3[3] = {ym, gy, yp};
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int a = 0; a < 3; ++a) T9[b][a] = (uint32_t)tile_major_index(0, xs3[a], ys3[b], 0, g) * ES;
  }

  // one z-iteration: collide plane z0 + j held in `cur`, load plane z + D into `nxt`
  // One z-iteration: collide plane z0 + j held in `cur`; load plane
  // z0 + j + D + LEAD - 1 into `ld`, `ldh`; publish plane z0 + j + D from
  // `pub`, `pubh` (the same buffers when LEAD = 1).
  auto iteration = [&](int j, real (&cur)[Q], real (&ld)[Q], real (&ldh)[Q], real (&pub)[Q], real (&pubh)[Q]) {
    const int z = z0 + j;
    const bool more = j + D <= zlen;  // psi of plane z + D is needed by a later collision
    // ---- A: issue the loads of plane z + D + LEAD - 1 ----
    if (j + D + LEAD - 1 <= zlen) load_plane(j + D + LEAD - 1, ld, ldh);
    __asm__ volatile("" ::: "memory");

    // ---- B: collide plane z ----
    const int sm = slot(z - 1), s0 = slot(z), sp = slot(z + 1);
    const int par = xslot(z);
    bool here_solid = false;
    if constexpr (SOLID) here_solid = ring_solid[s0][ly + 1][lx + 1] != 0;
    const real rhoA = xch[par][0][0][ly][lx], rhoB = xch[par][1][0][ly][lx];
    const real rho_k = k == 0 ? rhoA : rhoB;
    // float arithmetic: one reciprocal and fused products (this kernel
    // serves float32 and float16-shifted storage only)
    const real inv_den = real(1) / fmaf(omA, rhoA, omB * rhoB);
    real up[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) up[a] = fmaf(omA, xch[par][0][1 + a][ly][lx], omB * xch[par][1][1 + a][ly][lx]) * inv_den;
    // S = sum_i w_i psi(x + c_i) c_i, by weight class: sum the unit-weight
    // differences first, then scale once per class
    real S1[3] = {real(0), real(0), real(0)}, S2[3] = {real(0), real(0), real(0)};
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const int si = CZ[i] < 0 ? sm : (CZ[i] > 0 ? sp : s0);
      const real p = ring[si][1 - k][ly + 1 + CY[i]][lx + 1 + CX[i]];
      real (&Sw)[3] = i < 7 ? S1 : S2;
      if (CX[i] == 1) Sw[0] = Sw[0] + p;
      if (CX[i] == -1) Sw[0] = Sw[0] - p;
      if (CY[i] == 1) Sw[1] = Sw[1] + p;
      if (CY[i] == -1) Sw[1] = Sw[1] - p;
      if (CZ[i] == 1) Sw[2] = Sw[2] + p;
      if (CZ[i] == -1) Sw[2] = Sw[2] - p;
    }
    const real psi_k = ring[s0][k][ly + 1][lx + 1];
    const real ratio = rho_k == real(0) ? real(1) : psi_k / rho_k;
    const real ak = tgk * ratio;
    real v[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) v[a] = fmaf(-ak, fmaf(weight<real>(1), S1[a], weight<real>(7) * S2[a]), up[a]);
    const real vx = v[0], vy = v[1], vz = v[2];
    if constexpr (RECORD) {
      if (active) {
        const size_t node = row + plane_n * (uint32_t)z;
        const size_t Nn = (size_t)g.N;
        rec[(size_t)k * Nn + node] = here_solid ? real(0) : rho_k;
#pragma unroll
        for (int a = 0; a < 3; ++a) rec[(size_t)(2 + 3 * k + a) * Nn + node] = here_solid ? real(0) : xch[par][k][1 + a][ly][lx];
        rec[(size_t)(8 + k) * Nn + node] = psi_k;
      }
    }
    if (active && !here_solid) {
      const uint32_t Z[3] = {plane_n * (uint32_t)wrapz(z - 1), plane_n * (uint32_t)z, plane_n * (uint32_t)wrapz(z + 1)};
      const uint32_t here = row + Z[1];
      real fs_all[Q];
      relax_f32(cur, fs_all, rho_k, vx, vy, vz, omk, omck);
      if constexpr (TILED && !SOLID) {
        // every store of direction i goes to one z-plane and one population
        // row block: uniform descriptor and scalar offset, lane offset T9
        const __amdgpu_buffer_rsrc_t rz[3] = {zplane(fout, wrapz(z - 1)), zplane(fout, z), zplane(fout, wrapz(z + 1))};
#pragma unroll
        for (int i = 0; i < Q; ++i)
          buffer_store<ST>(encode<ST>(fs_all[i], c.shift[k][i]), rz[CZ[i] + 1], T9[CY[i] + 1][CX[i] + 1],
                           (uint32_t)(k * Q + i) * kRowBlock);
      } else {
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const real fs = fs_all[i];
        uint32_t dn = X[CX[i] + 1] + Y[CY[i] + 1] + Z[CZ[i] + 1];
        int di = i;
        if constexpr (SOLID) {
          if (i != 0) {
            const int si = CZ[i] < 0 ? sm : (CZ[i] > 0 ? sp : s0);
            if (ring_solid[si][ly + 1 + CY[i]][lx + 1 + CX[i]]) {
              dn = here;
              di = OPP[i];
            }
          }
        }
        if constexpr (TILED) {
          // bounce-back (di != i) lands in this node's own slot di
          const bool own = SOLID && di != i;
          const int zz = own ? z : (CZ[i] < 0 ? wrapz(z - 1) : (CZ[i] > 0 ? wrapz(z + 1) : z));
          char* zb = reinterpret_cast<char*>(fout) + (size_t)zz * zbytes + (size_t)(k * Q + di) * kRowBlock;
          *reinterpret_cast<store*>(zb + (own ? T9[1][1] : T9[CY[i] + 1][CX[i] + 1])) = encode<ST>(fs, c.shift[k][i]);
        } else {
          *reinterpret_cast<store*>(ok + (size_t)di * pbytes + dn * ES) = encode<ST>(fs, c.shift[k][i]);
        }
      }
      }
    }

    // ---- C: psi and exchange of plane z + D ----
    if (more) publish(z + D, pub, pubh);
    lds_barrier();
  };
  constexpr int PERIOD = NB % LEAD == 0 ? NB : NB * LEAD;
  for (int j0 = 0; j0 < zlen; j0 += PERIOD) {
#pragma unroll
    for (int u = 0; u < PERIOD; ++u)
      if (j0 + u < zlen)
        iteration(j0 + u, buf[u % NB], buf[(u + D + LEAD - 1) % NB], hbuf[(u + D + LEAD - 1) % LEAD],
                  buf[(u + D) % NB], hbuf[(u + D) % LEAD]);
  }
}

// Owner map of moving particles: the particle index at solid nodes; at fluid
// nodes kOwnerFluid, or kOwnerNear within R + 1.5 of a centre (every fluid
// end of a link lies within R + sqrt 2), where the fluid step records the
// density for the particles' link pass.
constexpr int kOwnerFluid = 0x7fffffff;
constexpr int kOwnerNear = 0x7ffffffe;  // fluid, possibly next to a particle

__device__ __forceinline__ bool owner_fluid(int o) { return o >= kOwnerNear; }

// Particle coupling of the colour-gradient pair kernel (PART): the owner map
// of the current positions and the float64 densities [2][N] that fluid nodes
// near a particle record for the link pass.
struct PartFluid {
  const int* owner;
  double* rho;
};

// ---------------------------------------------------------------------------
// Component-pair variant (float64 Shan-Chen; every colour-gradient step).
// Each wave holds 32 nodes of one tile row for both components: lanes 0..31
// carry component A, lanes 32..63 component B of the same nodes, and the
// partner lane (lane ^ 32) supplies the other component's density and
// momentum by a lane shuffle.  A tile row of TX = 32 or 64 nodes takes
// TX / 32 waves.  Ring of three planes of the stencil field: psi of both
// components (MODEL = kModelSC) or the phase field (kModelCG, whose
// recolouring also needs the partner's 19 post-perturbation populations,
// one shuffle each).
//
// STAGED = false: no prefetch.  The plane z + 1 loads go to registers and
// are consumed in the same iteration, which keeps the float64 register
// budget (two planes of 19 populations) within 256 VGPRs without spilling,
// but leaves their latency exposed.
//
// STAGED = true (float64 storage, nx a multiple of TX, no solids): the
// populations of plane z + 2 -- the tile's rows -1 .. TY and its two side
// columns, both components -- are copied from HBM straight into an LDS
// stage by direct-to-LDS loads (global_load_lds, which bypass the
// registers), issued before plane z is collided and waited for after its
// stores.  Their latency hides behind a whole collision without costing a
// register.  After the wait, psi of plane z + 2 is formed from the stage and
// the plane's interior populations move into registers for its own
// collision two iterations later.  Stage: 38 population planes x ((TY + 2)
// rows x TX nodes + 2 (TY + 2) side nodes) float64: 120,384 bytes for
// 64 x 4 tiles, 103,360 for 32 x 8, so one workgroup per compute unit.
// ---------------------------------------------------------------------------
//
// TILED: the populations are in the tile-major layout (64 x 4 tiles, no
// fixed solids, either model); only the addressing differs.
//
// PART (colour gradient with moving particles, unstaged; structure of arrays
// or, TILED, the tile-major layout): the solid nodes are those the owner map
// gives to a particle.
// Neutral wetting: in the phase-field stencil of a fluid node, a neighbour
// inside a particle contributes the node's own Theta.  Streaming is blind:
// every fluid node pushes its 19 post-collision populations to x + c_i and
// every solid node pushes zeros, so that the particles' link pass finds the
// population sent into a particle waiting in the particle node's slot (and
// the zero it replaces in the fluid node's).  Fluid nodes near a particle
// record rho_A and rho_B for that pass.
//
// The float32 particle kernel on the tile-major layout is held to 128
// registers (four waves per SIMD, two workgroups per compute unit); it needs
// 153 unconstrained, which leaves one workgroup per compute unit.
template <int ST, bool SOLID, int TY, bool RECORD, bool STAGED, int TX = kFusedTX, int MODEL = kModelSC,
          bool TILED = false, bool PART = false>
__global__ void __launch_bounds__(2 * TX * TY, (PART && TILED && sizeof(store_t<ST>) == 4) ? 4 : 1)
    k_fused_pair(const store_t<ST>* __restrict__ fin, store_t<ST>* __restrict__ fout,
                 const uint8_t* __restrict__ mask, Geometry g, StepCoeffs c, FusedTiling t,
                 real_t<ST>* __restrict__ rec, PartFluid pf = {}) {
  using real = real_t<ST>;
  constexpr int WPR = TX / 32;  // waves per tile row
  constexpr int NW = TY * WPR;  // waves per workgroup
  constexpr int RX = TX + 2, RY = TY + 2;
  static_assert(TX == 32 || TX == 64, "a wave carries 32 nodes of a row");
  static_assert(2 * (2 * RX + 2 * TY) <= 64 * NW, "too few lanes for the halo tasks");
  static_assert(!STAGED || (sizeof(store_t<ST>) == 8 && TY % 2 == 0 && 4 * (TY + 2) <= 64),
                "the stage layout assumes float64, and one wave covers the side columns");
  // With solids the staged variant needs more than the 256 registers two
  // waves per SIMD allow and spills; the unstaged kernel is faster there.
  static_assert(!(STAGED && SOLID), "lattices with solids run the unstaged kernel");
  static_assert(MODEL == kModelSC || (!RECORD && (!SOLID || PART)),
                "the colour-gradient step has no adjoint record, and solids only as particles");
  static_assert(!PART || (SOLID && MODEL == kModelCG && !STAGED && sizeof(store_t<ST>) >= 4),
                "particles: colour gradient, unstaged, float32 or float64 storage");
  static_assert(!TILED || (TX == kTileX && TY % kTileY == 0 && (!SOLID || PART)),
                "the tile-major layout serves the 64-wide step without solids or record");
  constexpr int NQ = ((TY + 2) * TX / 2 + 63) / 64;  // 16-byte loads per lane covering one population plane's rows
  __shared__ real ring[3][2][RY][RX];
  // bit 0: solid; 2: fluid near a particle (PART)
  __shared__ uint8_t ring_solid[SOLID ? 3 : 1][SOLID ? RY : 1][SOLID ? RX : 1];
  constexpr int KI = 2 * Q;                      // population planes of both components
  constexpr int ST_ROWS = KI * RY * TX;          // [ki][row -1 .. TY][x] block
  constexpr int ST_SIDE = KI * 2 * RY;           // [ki][left rows -1 .. TY, right rows -1 .. TY]
  __shared__ real stage[STAGED ? ST_ROWS + ST_SIDE : 1];

  const int w = fused_work_item(blockIdx.x, t.total, t.per_round);
  const int chunk = w / (t.tiles_x * t.tiles_y);
  const int tile = w - chunk * (t.tiles_x * t.tiles_y);
  const int ty0 = (tile / t.tiles_x) * TY, tx0 = (tile % t.tiles_x) * TX;
  const int z0 = chunk * t.chunk;
  const int zlen = min(t.chunk, g.nz - z0);

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int k = lane >> 5;
  const int lx = (wave % WPR) * 32 + (lane & 31), ly = wave / WPR;
  const int gx = (tx0 + lx) % g.nx, gy = (ty0 + ly) % g.ny;
  const bool active = (tx0 + lx) < g.nx && (ty0 + ly) < g.ny;
  const long long row = (long long)gx + (long long)g.nx * gy;
  const long long plane_n = (long long)g.nx * g.ny;
  const long long kplane = (long long)(k * Q) * g.Npad;

  // halo task of this lane, if any: node h of the ring's border, component hk
  const int nh = 2 * RX + 2 * TY;
  const int task = threadIdx.x;
  const bool has_halo = task < 2 * nh;
  int hx = 0, hy = 0, hk = 0;
  if (has_halo) {
    const int h = task >> 1;
    hk = task & 1;
    if (h < RX) { hx = h - 1; hy = -1; }
    else if (h < 2 * RX) { hx = h - RX - 1; hy = TY; }
    else if (h < 2 * RX + TY) { hx = -1; hy = h - 2 * RX; }
    else { hx = TX; hy = h - 2 * RX - TY; }
  }
  const int hgx = ((tx0 + hx) % g.nx + g.nx) % g.nx;
  const int hgy = ((ty0 + hy) % g.ny + g.ny) % g.ny;
  const long long hrow = (long long)hgx + (long long)g.nx * hgy;
  const long long hkplane = (long long)(hk * Q) * g.Npad;

  auto wrapz = [&](int z) { return z < 0 ? z + g.nz : (z >= g.nz ? z - g.nz : z); };

  // ---- direct-to-LDS staging (STAGED only) ----
  // Byte offsets within one z-plane of a population plane.  Rows: chunk
  // c = 64 q + lane (c < RY TX / 2) covers row c / (TX / 2) - 1 of the tile
  // and x = 2 (c % (TX / 2)) and the next node (16 bytes).  Sides: lane <
  // 4 RY covers one half of the float64 at side node lane / 2 (left column
  // for < RY, right column after, rows -1 .. TY).
  uint32_t voff16[NQ] = {}, voff4 = 0;
  bool on16[NQ] = {}, on4 = false;
  int ibase = 0, hbase = 0;  // stage index of value 0 of this lane's interior node and halo node
  bool hrows = false;        // halo node in a stage row (else in a side column)
  if constexpr (STAGED) {
    auto wrapy = [&](int y) { return ((y % g.ny) + g.ny) % g.ny; };  // y may be off by more than ny when ny < TY
    // element offset of node (x, y) within population plane 0 of a z-plane
    auto in_plane = [&](int x, int y) -> uint32_t {
      if constexpr (TILED) return (uint32_t)tile_major_index(0, x, y, 0, g);
      else return (uint32_t)x + (uint32_t)g.nx * (uint32_t)y;
    };
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int cq = 64 * q + lane;
      on16[q] = cq < RY * (TX / 2);
      const int r = cq / (TX / 2), xp = cq % (TX / 2);
      voff16[q] = in_plane(tx0 + 2 * xp, wrapy(ty0 + r - 1)) * 8u;  // x even: both nodes in one tile row
    }
    on4 = lane < 4 * RY;
    {
      const int sn = lane >> 1, r = sn % RY;
      const int sx = sn < RY ? (tx0 == 0 ? g.nx - 1 : tx0 - 1) : (tx0 + TX == g.nx ? 0 : tx0 + TX);
      voff4 = in_plane(sx, wrapy(ty0 + r - 1)) * 8u + 4u * (uint32_t)(lane & 1);
    }
    ibase = (k * Q * RY + ly + 1) * TX + lx;
    hrows = hx >= 0 && hx < TX;
    hbase = hrows ? (hk * Q * RY + hy + 1) * TX + hx : ST_ROWS + hk * Q * 2 * RY + (hx < 0 ? 0 : RY) + hy + 1;
  }
  // Issue the loads of plane zz into the stage.  Wave w copies population
  // planes ki = w, w + NW, ... (uniform per wave).
  auto stage_issue = [&](int zz) {
    typedef __attribute__((address_space(3))) void lds_void;
    typedef __attribute__((address_space(1))) void glb_void;
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    const size_t zstride = TILED ? (size_t)KI * (size_t)plane_n : (size_t)plane_n;  // elements per z-plane
    const size_t kstride = TILED ? (size_t)kTileNodes : (size_t)g.Npad;              // ... per population plane
    const char* zbase = reinterpret_cast<const char*>(fin) + zstride * (size_t)zz * 8u;
#pragma unroll
    for (int m = 0; m < (KI + NW - 1) / NW; ++m) {
      const int ki = wv + NW * m;
      if (ki < KI) {
        const char* base = zbase + (size_t)ki * kstride * 8u;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
          if (on16[q])
            __builtin_amdgcn_global_load_lds((glb_void*)(base + voff16[q]),
                                             (lds_void*)(&stage[ki * RY * TX + 128 * q]), 16, 0, 0);
        if (on4) __builtin_amdgcn_global_load_lds((glb_void*)(base + voff4), (lds_void*)(&stage[ST_ROWS + ki * 2 * RY]), 4, 0, 0);
      }
    }
  };

  auto rho_of = [&](long long n, long long kp, int kk, real (&v)[Q]) -> real {
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i] = decode<ST>(fin[kp + (long long)i * g.Npad + n], c.shift[kk][i]);
    return density<real>(v);
  };
  // Ring entry of a node from its density rho_kk.  Shan-Chen: psi_kk (0 at
  // solid nodes).  Colour gradient: the phase field
  // Theta = (rho_A - rho_B) / (rho_A + rho_B), written by the component-A
  // lane; the lane holding component B of the same node is lane ^ pm, and
  // both lanes must reach this call.
  auto ring_put = [&](int s, int kk, int y, int x, real rho, bool solid, int pm) {
    if constexpr (MODEL == kModelSC) {
      ring[s][kk][y][x] = (SOLID && solid) ? real(0) : pseudopotential(rho, coef_ref<real>(c));
    } else {
      const real o = pm == 32 ? other_half(rho) : __shfl_xor(rho, pm, 64);
      if (kk == 0) ring[s][0][y][x] = (SOLID && solid) ? real(0) : (rho - o) / (rho + o);
    }
  };

  auto rho_tiled = [&](int x, int y, int z, int kk, real (&v)[Q]) -> real {
    const long long t = tile_major_index(kk * Q, x, y, z, g);
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i] = decode<ST>(fin[t + (long long)i * kTileNodes], c.shift[kk][i]);
    return density<real>(v);
  };

  // ring slot s <- plane z; interior lanes keep their populations in `keep`
  auto fill = [&](int s, int z, real (&keep)[Q]) {
    const long long zoff = plane_n * z;
    {
      const long long n = row + zoff;
      bool solid = false, near = false;
      if constexpr (PART) {
        const int o = pf.owner[n];
        solid = !owner_fluid(o);
        near = o == kOwnerNear;
      } else if constexpr (SOLID) {
        solid = mask[n] != 0;
      }
      const real rho = TILED ? rho_tiled(gx, gy, z, k, keep) : rho_of(n, kplane, k, keep);
      ring_put(s, k, ly + 1, lx + 1, rho, solid, 32);
      if constexpr (SOLID) if (k == 0) ring_solid[s][ly + 1][lx + 1] = solid ? 1 : (near ? 2 : 0);
    }
    if (has_halo) {
      const long long n = hrow + zoff;
      bool solid = false;
      if constexpr (PART) solid = !owner_fluid(pf.owner[n]);
      else if constexpr (SOLID) solid = mask[n] != 0;
      real tmp[Q];
      const real rho = TILED ? rho_tiled(hgx, hgy, z, hk, tmp) : rho_of(n, hkplane, hk, tmp);
      ring_put(s, hk, hy + 1, hx + 1, rho, solid, 1);
      if constexpr (SOLID) if (hk == 0) ring_solid[s][hy + 1][hx + 1] = solid;
    }
  };

  // Two population buffers swap roles every plane (the loop below is
  // unrolled by two): `cur` holds plane z while it is collided, `nxt` plane
  // z + 1; once plane z is stored, its registers take plane z + 2 (STAGED)
  // or the loads of the next plane go to the other buffer.
  real bufA[Q], bufB[Q];
  fill(0, wrapz(z0 - 1), bufB);  // populations of plane z0 - 1 are not needed
  fill(1, z0, bufA);
  if constexpr (STAGED) fill(2, wrapz(z0 + 1), bufB);
  __syncthreads();

  // TILED: in-plane byte offsets of this lane's nine (x +- 1, y +- 1)
  // destinations in its component's population block, for push stores by
  // raw buffer (descriptor of the z-plane, scalar offset of the population)
  uint32_t P9[3][3] = {};
  const size_t zbytes = (size_t)KI * (size_t)plane_n * sizeof(store_t<ST>);  // < 2^32 where TILED (host check)
  if constexpr (TILED) {
    const int xs3[3] = {gx == 0 ? g.nx - 1 : gx - 1, gx, gx == g.nx - 1 ? 0 : gx + 1};
    const int ys3[3] = {gy == 0 ? g.ny - 1 : gy - 1, gy, gy == g.ny - 1 ? 0 : gy + 1};
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int a = 0; a < 3; ++a)
        P9[b][a] = (uint32_t)tile_major_index(k * Q, xs3[a], ys3[b], 0, g) * (uint32_t)sizeof(store_t<ST>);
  }
  auto zplane = [&](int z) {
    return buffer_rsrc(reinterpret_cast<const char*>(fout) + (size_t)z * zbytes, (uint32_t)zbytes);
  };

  const real omk = coef_om<real>(c, k), omck = coef_omc<real>(c, k), tgk = coef_tg<real>(c, k);
  const real omA = coef_om<real>(c, 0), omB = coef_om<real>(c, 1);

  // Post-collision populations of plane z of this lane's node to their
  // destinations in fout (push streaming; bit i of bb: bounce-back).
  auto push_plane = [&](int z, const real (&fs)[Q], uint32_t bb) {
    const int zm = wrapz(z - 1), zp = wrapz(z + 1);
    const int xm = gx == 0 ? g.nx - 1 : gx - 1, xp = gx == g.nx - 1 ? 0 : gx + 1;
    const int ym = gy == 0 ? g.ny - 1 : gy - 1, yp = gy == g.ny - 1 ? 0 : gy + 1;
    const int X[3] = {xm, gx, xp};
    const int Y[3] = {ym, gy, yp};
    const int Z[3] = {zm, z, zp};
    const long long here = row + plane_n * z;
    if constexpr (TILED) {
      const __amdgpu_buffer_rsrc_t rz[3] = {zplane(zm), zplane(z), zplane(zp)};
      constexpr uint32_t kRowBlock = (uint32_t)kTileNodes * (uint32_t)sizeof(store_t<ST>);
#pragma unroll
      for (int i = 0; i < Q; ++i)
        buffer_store<ST>(encode<ST>(fs[i], c.shift[k][i]), rz[CZ[i] + 1], P9[CY[i] + 1][CX[i] + 1],
                         (uint32_t)i * kRowBlock);
      return;
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      long long dst;
      if constexpr (TILED) {
        dst = tile_major_index(k * Q + i, X[CX[i] + 1], Y[CY[i] + 1], Z[CZ[i] + 1], g);
      } else {
        dst = kplane + (long long)i * g.Npad + X[CX[i] + 1] +
              (long long)g.nx * (Y[CY[i] + 1] + (long long)g.ny * Z[CZ[i] + 1]);
      }
      if constexpr (SOLID)
        if ((bb >> i) & 1u) dst = kplane + (long long)OPP[i] * g.Npad + here;
      fout[dst] = encode<ST>(fs[i], c.shift[k][i]);
    }
  };
  auto iteration = [&](int j, real (&cur)[Q], real (&nxt)[Q]) {
    const int z = z0 + j;
    const int sm = j % 3, s0 = (j + 1) % 3, sp = (j + 2) % 3;  // ring slots of planes z-1, z, z+1
    // STAGED: plane z + 2 is loaded while plane z is collided; its psi is
    // needed unless z + 1 is the chunk's far neighbour plane.
    const bool more = j + 2 <= zlen;
    if constexpr (STAGED) {
      if (more) stage_issue((z + 2) % g.nz);
    } else {
      fill(sp, wrapz(z + 1), nxt);
      __syncthreads();
    }

    bool here_solid = false;
    if constexpr (SOLID) here_solid = (ring_solid[s0][ly + 1][lx + 1] & 1) != 0;
    const real rho_k = density<real>(cur);
    real m_k[3] = {lattice_sum<0, 0, real>(cur), lattice_sum<1, 0, real>(cur), lattice_sum<2, 0, real>(cur)};
    const real rho_o = other_half(rho_k);
    real m_o[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) m_o[a] = other_half(m_k[a]);
    const real rhoA = k == 0 ? rho_k : rho_o, rhoB = k == 0 ? rho_o : rho_k;
    const real den = omA * rhoA + omB * rhoB;
    real up[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const real mA = k == 0 ? m_k[a] : m_o[a], mB = k == 0 ? m_o[a] : m_k[a];
      up[a] = (omA * mA + omB * mB) / den;
    }
    // S = sum_i w_i q(x + c_i) c_i, q = psi of the other component
    // (Shan-Chen) or the phase field (colour gradient; with particles a
    // neighbour inside one gives this node's own phase field)
    constexpr bool SC = MODEL == kModelSC;
    real S[3] = {real(0), real(0), real(0)};
    [[maybe_unused]] const real theta_here = ring[s0][0][ly + 1][lx + 1];
    // PART: bit i set where neighbour x + c_i is solid.  Only a node near a
    // particle can have one (a fluid node beside a particle node lies within
    // R + sqrt 2 of its centre), so the other waves skip the flag reads.
    [[maybe_unused]] uint32_t solid_nb = 0;
    if constexpr (PART) {
      if (ring_solid[s0][ly + 1][lx + 1] == 2) {
#pragma unroll
        for (int i = 1; i < Q; ++i) {
          const int si = CZ[i] < 0 ? sm : (CZ[i] > 0 ? sp : s0);
          if (ring_solid[si][ly + 1 + CY[i]][lx + 1 + CX[i]] & 1) solid_nb |= 1u << i;
        }
      }
    }
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const int si = CZ[i] < 0 ? sm : (CZ[i] > 0 ? sp : s0);
      real q = ring[si][SC ? 1 - k : 0][ly + 1 + CY[i]][lx + 1 + CX[i]];
      if constexpr (PART)
        if ((solid_nb >> i) & 1u) q = theta_here;
      const real tt = weight<real>(i) * q;
      if (CX[i] == 1) S[0] = S[0] + tt;
      if (CX[i] == -1) S[0] = S[0] - tt;
      if (CY[i] == 1) S[1] = S[1] + tt;
      if (CY[i] == -1) S[1] = S[1] - tt;
      if (CZ[i] == 1) S[2] = S[2] + tt;
      if (CZ[i] == -1) S[2] = S[2] - tt;
    }
    const real psi_k = ring[s0][k][ly + 1][lx + 1];
    const real ratio = rho_k == real(0) ? real(1) : psi_k / rho_k;
    const real ak = tgk * ratio;
    const real vx = up[0] - ak * S[0];
    const real vy = up[1] - ak * S[1];
    const real vz = up[2] - ak * S[2];
    const real vv = (vx * vx + vy * vy) + vz * vz;
    const real t15 = real(1.5) * vv;
    if constexpr (PART) {
      if (active && ring_solid[s0][ly + 1][lx + 1] == 2) pf.rho[(long long)k * g.N + row + plane_n * z] = double(rho_k);
    }
    if constexpr (RECORD) {
      if (active) {
        const long long node = row + plane_n * z;
        rec[(long long)k * g.N + node] = here_solid ? real(0) : rho_k;
#pragma unroll
        for (int a = 0; a < 3; ++a) rec[(long long)(2 + 3 * k + a) * g.N + node] = here_solid ? real(0) : m_k[a];
        rec[(long long)(8 + k) * g.N + node] = psi_k;
      }
    }

    // Post-collision populations.  STAGED keeps them in `cur` (and the
    // bounce-back directions in a bit mask, since ring slot sm is refilled
    // before they are stored) and stores them after the stage wait, so that
    // the stores drain during the next collision instead of delaying the wait.
    uint32_t bounced = 0;
    auto push = [&](const real (&fs)[Q], uint32_t bb) { push_plane(z, fs, bb); };
    if (active && !here_solid) {
      real fs[Q];
      if constexpr (SC) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const real cu = cdot<real>(i, vx, vy, vz);
          const real feq = (weight<real>(i) * rho_k) * (((real(1) + real(3) * cu) + real(4.5) * cu * cu) - t15);
          fs[i] = omck * cur[i] + omk * feq;
          if constexpr (SOLID) {
            if (i != 0) {
              const int si = CZ[i] < 0 ? sm : (CZ[i] > 0 ? sp : s0);
              if (ring_solid[si][ly + 1 + CY[i]][lx + 1 + CX[i]] & 1) bounced |= 1u << i;
            }
          }
        }
      } else {
        // Colour gradient (Appendix): BGK with the mean-viscosity omega plus
        // the perturbation, per component; the two summed into f*; f* split
        // between the components by the recolouring.  The partner lane
        // (lane ^ 32, same node, other component) is active exactly when
        // this lane is, so the exchanges below are complete.
        //
        // float64 keeps the oracle's operations (and so its bits).  float
        // arithmetic takes hardware reciprocals and square root (about 1 ulp)
        // and multiplies by them: three reciprocals per node instead of 28
        // correctly rounded quotients, most of this step's vector ALU work.
        constexpr bool F32 = sizeof(real) == 4;
        const real rho = rhoA + rhoB;
        [[maybe_unused]] real inv_rho = real(0);
        if constexpr (F32) inv_rho = __builtin_amdgcn_rcpf(rho);
        real u[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const real mA = k == 0 ? m_k[a] : m_o[a], mB = k == 0 ? m_o[a] : m_k[a];
          if constexpr (F32) u[a] = (mA + mB) * inv_rho;
          else u[a] = (mA + mB) / rho;
        }
        const real g3[3] = {real(3) * S[0], real(3) * S[1], real(3) * S[2]};
        const real gg = (g3[0] * g3[0] + g3[1] * g3[1]) + g3[2] * g3[2];
        const bool iface = gg > cg_interface_g2<real>();
        real gn = real(0), nv[3];
        if constexpr (F32) {
          gn = iface ? __builtin_amdgcn_sqrtf(gg) : real(0);
          const real inv_gn = iface ? __builtin_amdgcn_rcpf(gn) : real(0);
#pragma unroll
          for (int a = 0; a < 3; ++a) nv[a] = g3[a] * inv_gn;
        } else {
          gn = iface ? real(sqrt(gg)) : real(0);
#pragma unroll
          for (int a = 0; a < 3; ++a) nv[a] = iface ? g3[a] / gn : real(0);
        }
        real om, r, ck;
        if constexpr (F32) {
          // omega = 2 / (6 nubar + 1) = 2 (1/nubar) / (6 + 1/nubar)
          const real inv_nubar = (rhoA * inv_rho) * coef_cg_inv_nu<real>(c, 0) + (rhoB * inv_rho) * coef_cg_inv_nu<real>(c, 1);
          om = (real(2) * inv_nubar) * __builtin_amdgcn_rcpf(real(6) + inv_nubar);
          r = (coef_cg_beta<real>(c) * (rhoA * rhoB)) * (inv_rho * inv_rho);
          ck = rho_k * inv_rho;
        } else {
          const real inv_nubar = (rhoA / rho) * coef_cg_inv_nu<real>(c, 0) + (rhoB / rho) * coef_cg_inv_nu<real>(c, 1);
          const real nubar = real(1) / inv_nubar;
          om = real(2) / (real(6) * nubar + real(1));
          r = (coef_cg_beta<real>(c) * (rhoA * rhoB)) / (rho * rho);
          ck = rho_k / rho;
        }
        const real pcoef = (real(0.5) * (coef_cg_s225<real>(c) * om)) * gn;
        const real uu = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
        const real t15u = real(1.5) * uu;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const real cu = cdot<real>(i, u[0], u[1], u[2]);
          const real feq = (weight<real>(i) * rho_k) * (((real(1) + real(3) * cu) + real(4.5) * cu * cu) - t15u);
          const real cn = cdot<real>(i, nv[0], nv[1], nv[2]);
          const real pert = pcoef * (weight<real>(i) * (cn * cn) - cg_b<real>(i));
          const real fk = (cur[i] + om * (feq - cur[i])) + pert;
          const real fo = other_half(fk);
          const real fstar = k == 0 ? fk + fo : fo + fk;
          const real cosphi = F32 ? cn * (real(1) / cg_clen<real>(i)) : cn / cg_clen<real>(i);
          const real t = (r * cosphi) * (weight<real>(i) * rho);
          fs[i] = k == 0 ? ck * fstar + t : ck * fstar - t;
        }
      }
      if constexpr (STAGED) {
#pragma unroll
        for (int i = 0; i < Q; ++i) cur[i] = fs[i];
      } else {
        push(fs, bounced);
      }
    }
    if constexpr (PART) {
      if (active && here_solid) {
        real zero[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) zero[i] = real(0);
        push(zero, 0u);
      }
    }
    // psi of the halo node of plane z + 2 from the stage into ring slot sm
    auto drain_halo = [&]() {
      if (has_halo) {
        // constant strides, so that every read is one base register plus an immediate offset
        real h[Q];
        if (hrows) {
#pragma unroll
          for (int i = 0; i < Q; ++i) h[i] = stage[hbase + i * RY * TX];
        } else {
#pragma unroll
          for (int i = 0; i < Q; ++i) h[i] = stage[hbase + i * 2 * RY];
        }
        ring_put(sm, hk, hy + 1, hx + 1, density<real>(h), false, 1);
      }
    };
    if constexpr (STAGED) {
      const bool store = active && !here_solid;
      if (more) {
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's stage loads have landed
        lds_barrier();                        // ... and every other wave's; ring slot sm is free
        drain_halo();
        if (store) push(cur, bounced);
#pragma unroll
        for (int i = 0; i < Q; ++i) cur[i] = stage[ibase + i * RY * TX];  // plane z + 2
        ring_put(sm, k, ly + 1, lx + 1, density<real>(cur), false, 32);
      } else {
        if (store) push(cur, bounced);
      }
      lds_barrier();  // psi of z + 2 visible; the stage may be refilled
    } else {
      // A full barrier here measured faster than an LDS-only one: the wave
      // then issues its next loads only after its stores have drained.
      __syncthreads();
    }
  };
  for (int j0 = 0; j0 < zlen; j0 += 2) {
    iteration(j0, bufA, bufB);
    if (j0 + 1 < zlen) iteration(j0 + 1, bufB, bufA);
  }
}

}  // namespace lbd
