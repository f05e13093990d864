// Moving rigid spheres in the single-fluid step and in the two-component
// colour-gradient step: the paper's particle solver (Sec. 2, Eq. PARDYN with
// leap-frog; Sec. 3 step order; Appendix, Eqs. UPI, LADDFLBE, FORCEPP,
// FORCEPARTEQ, TORQUEPARTEQ), HIP kernels.
//
// One step, t -> t + 1 (each line one launch):
//   k1p_step         collide fluid nodes and push every population, solid
//                    nodes push zeros; fluid nodes near a particle record
//                    their density (two components: k_fused_pair with PART,
//                    which records rho_A and rho_B)
//   kp_force_move    one workgroup per particle: bounce-back at its links with
//                    the moving-wall correction W_i = 2 rho w_i (u_b . c_i) / c_s^2,
//                    u_b = v + omega x r_b; force and torque summed over the
//                    links in float64 in a fixed order; then the leap-frog
//                    update of velocity, angular velocity and position
//   kp_owner_fill,
//   kp_owner_scatter owner map of the new positions (lowest index wins)
//   kp_remap         one workgroup per particle: nodes covered by the move hand
//                    their momentum to the particle and are emptied; nodes
//                    uncovered start at f^eq(rho0, u_b) and take theirs from
//                    the particle
// Particle arithmetic (positions, surface velocities, W_i, forces) is
// float64 whatever the storage: the paper accumulates particle forces in
// double precision because the link terms cancel strongly.
//
// Two components (NC = 2): each component bounces back with its own
// density in the wall term, W^k_i = 2 rho^k w_i (u_b . c_i) / c_s^2, so that
// the pair carries the single-fluid term of the mixture density, and the
// particle receives the momentum of both components' links; covered nodes
// hand over both components, uncovered nodes start each component at
// f^eq(rho0_k, u_b).
//
// Fixed summation order of a particle's link and covering sums, so that
// they are reproducible bit for bit.  The particle's box has S nodes per axis
// from lo_a = floor(r_a - R) - 1, numbered b = j_x + S (j_y + S j_z).  Thread l
// of the particle's 256-thread workgroup takes b = l, l + 256, ... in order,
// and at each node directions i = 1..18 in order.  Each wave combines its 64
// sums by a butterfly, a_l <- a_l + a_(l xor s) for s = 32, 16, ..., 1; the
// four wave results give (A_0 + A_1) + (A_2 + A_3).
//
// Owner map: the particle index at solid nodes; at fluid nodes kOwnerFluid,
// or kOwnerNear within R + 1.5 of a centre (every fluid end of a link lies
// within R + sqrt 2), where the fluid kernel records the density.
#pragma once

#include "lb_fused.h"
#include "lb_kernels.h"

namespace lbd {

constexpr int kPartThreads = 256;

struct PartState {
  double* pos;     // [P][3], in [0, L)
  double* vel;     // [P][3], at half steps
  double* omg;     // [P][3], at half steps
  double* force;   // [P][3], of the last step
  double* torque;  // [P][3]
  int count;
  int box;         // S = floor(2R) + 4
  double radius, r2, near2, inner2, mass, inertia;  // R^2, (R + 1.5)^2, (R - 1.5)^2 or -1
  double rho0[2];  // density of each component at nodes the particles uncover
};

// Population plane ki of node n = x + nx (y + ny z): structure of arrays, or
// the tile-major layout of the fused steps (TILED).
template <bool TILED>
__device__ __forceinline__ long long pop_index(int ki, int n, int x, int y, int z, const Geometry& g) {
  if constexpr (TILED) return tile_major_index(ki, x, y, z, g);
  else return (long long)ki * g.Npad + n;
}

// Periodic wrap of any coordinate (a box of a particle whose state has gone
// non-finite still addresses the lattice).  A particle's box coordinates lie
// within one period of the lattice whenever it is at least R + 2 wide, so
// the remainder is only taken for the others.
__device__ __forceinline__ int wrap_coord(int c, int L) {
  if (c >= 0 && c < L) return c;
  if (c < 0 && c >= -L) return c + L;
  if (c >= L && c - L < L) return c - L;
  c %= L;
  return c < 0 ? c + L : c;
}

// Periodic wrap of a coordinate in [-1, L], a neighbour of a wrapped one.
__device__ __forceinline__ int wrap_step(int c, int L) { return c < 0 ? c + L : (c >= L ? c - L : c); }

// Nearest periodic image of a coordinate difference.
__device__ __forceinline__ double fold(double d, double L) {
  if (d > 0.5 * L) d = d - L;
  if (d < -0.5 * L) d = d + L;
  return d;
}

// One particle's centre, velocity and angular velocity, in registers.
struct PartRegs {
  double r[3], v[3], w[3];
};

__device__ __forceinline__ PartRegs part_regs(const PartState& ps, int p) {
  PartRegs q;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    q.r[a] = ps.pos[3 * p + a];
    q.v[a] = ps.vel[3 * p + a];
    q.w[a] = ps.omg[3 * p + a];
  }
  return q;
}

// Components of c_i for a direction known only at run time: the tables
// packed two bits per direction (component + 1).
constexpr unsigned long long pack_dirs(const int (&c)[Q]) {
  unsigned long long v = 0;
  for (int i = 0; i < Q; ++i) v |= (unsigned long long)(c[i] + 1) << (2 * i);
  return v;
}
constexpr unsigned long long kPackedCX = pack_dirs(CX), kPackedCY = pack_dirs(CY), kPackedCZ = pack_dirs(CZ);
__device__ __forceinline__ int cx_of(int i) { return int((kPackedCX >> (2 * i)) & 3ull) - 1; }
__device__ __forceinline__ int cy_of(int i) { return int((kPackedCY >> (2 * i)) & 3ull) - 1; }
__device__ __forceinline__ int cz_of(int i) { return int((kPackedCZ >> (2 * i)) & 3ull) - 1; }
__device__ __forceinline__ int opp_of(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// W_i and the link midpoint r_b (relative to the particle) for the link
// from fluid node (x, y, z) in direction i into the particle q.  c_i . u_b
// is summed in the order of cdot.
__device__ __forceinline__ double wall_term(int i, int x, int y, int z, double rho, const PartRegs& q,
                                            const Geometry& g, double (&rb)[3]) {
  const double* r = q.r;
  const double* v = q.v;
  const double* w = q.w;
  const int cx = cx_of(i), cy = cy_of(i), cz = cz_of(i);
  rb[0] = fold((double(x) + 0.5 * cx) - r[0], double(g.nx));
  rb[1] = fold((double(y) + 0.5 * cy) - r[1], double(g.ny));
  rb[2] = fold((double(z) + 0.5 * cz) - r[2], double(g.nz));
  const double ubx = v[0] + (w[1] * rb[2] - w[2] * rb[1]);
  const double uby = v[1] + (w[2] * rb[0] - w[0] * rb[2]);
  const double ubz = v[2] + (w[0] * rb[1] - w[1] * rb[0]);
  double cub = 0.0;
  if (cx == 1) cub = cub + ubx;
  if (cx == -1) cub = cub - ubx;
  if (cy == 1) cub = cub + uby;
  if (cy == -1) cub = cub - uby;
  if (cz == 1) cub = cub + ubz;
  if (cz == -1) cub = cub - ubz;
  return (6.0 * weight<double>(i)) * (rho * cub);
}

// decode / encode for the particle kernels' storages (float64 and float32
// keep no shift, so a run-time direction needs no table).
template <int ST>
__device__ __forceinline__ real_t<ST> decode_dir(store_t<ST> v) {
  static_assert(ST != ST_F16S, "particles run on float64 and float32 storage");
  return decode<ST>(v, 0.0f);
}
template <int ST>
__device__ __forceinline__ store_t<ST> encode_dir(real_t<ST> v) {
  static_assert(ST != ST_F16S, "particles run on float64 and float32 storage");
  return encode<ST>(v, 0.0f);
}

// Single-fluid step with particles.  One work-item per node, as k1_step.
// Every node pushes all 19 populations without looking at its neighbours:
// a fluid node its post-collision values, a solid node zeros.  A population
// pushed into a particle node therefore waits in that node's slot, and the
// slot of the fluid node it should bounce back into holds the zero its solid
// neighbour pushed; kp_force_move turns each such pair into the bounce-back
// with the moving-wall term.  Each slot has one writer.  Fluid nodes near a
// particle (kOwnerNear) record their density for that pass.
template <int ST>
__global__ void __launch_bounds__(kBlock) k1p_step(const store_t<ST>* __restrict__ fin, store_t<ST>* __restrict__ fout,
                                                   const int* __restrict__ owner, double* __restrict__ rho_buf,
                                                   Geometry g, StepCoeffs c) {
  using real = real_t<ST>;
  const int b = fused_work_item(blockIdx.x, gridDim.x, gridDim.x);
  const int n = b * kBlock + threadIdx.x;
  if (n >= g.N) return;
  const int own = owner[n];
  int x, y, z;
  node_xyz(n, g, x, y, z);
  int nb[Q];
  neighbours(x, y, z, g, nb);
  // Solid nodes hold zero populations; they go through the same arithmetic
  // (0/0 included) and store zeros in the same store instructions as the
  // fluid nodes of their wave.
  const bool solid = !owner_fluid(own);
  real f[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) f[i] = decode<ST>(fin[(long long)i * g.Npad + n], c.shift[0][i]);
  const real rho = density<real>(f);
  const real ux = lattice_sum<0, 0, real>(f) / rho;
  const real uy = lattice_sum<1, 0, real>(f) / rho;
  const real uz = lattice_sum<2, 0, real>(f) / rho;
  real fs[Q];
  if constexpr (sizeof(real) == 8) {
    const real om = coef_om<real>(c, 0), omc = coef_omc<real>(c, 0);
    const real t15 = real(1.5) * ((ux * ux + uy * uy) + uz * uz);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const real cu = cdot<real>(i, ux, uy, uz);
      const real feq = (weight<real>(i) * rho) * (((real(1) + real(3) * cu) + real(4.5) * cu * cu) - t15);
      fs[i] = omc * f[i] + om * feq;
    }
  } else {
    relax_f32(f, fs, rho, ux, uy, uz, coef_om<real>(c, 0), coef_omc<real>(c, 0));
  }
#pragma unroll
  for (int i = 0; i < Q; ++i)
    fout[(long long)i * g.Npad + nb[i]] = solid ? store_t<ST>(0) : encode<ST>(fs[i], c.shift[0][i]);
  if (own == kOwnerNear) rho_buf[n] = static_cast<double>(rho);
}

__device__ __forceinline__ double wave_sum_xor(double v) {
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) v = v + __shfl_xor(v, s, 64);
  return v;
}

// Box node b of a particle at r: unwrapped coordinates and the wrapped node index.
__device__ __forceinline__ int box_node(int b, const int (&lo)[3], int S, const Geometry& g, int (&cc)[3]) {
  cc[0] = lo[0] + b % S;
  cc[1] = lo[1] + (b / S) % S;
  cc[2] = lo[2] + b / (S * S);
  return wrap_coord(cc[0], g.nx) + g.nx * (wrap_coord(cc[1], g.ny) + g.ny * wrap_coord(cc[2], g.nz));
}

// Box coordinates of the nodes b, b + step, b + 2 step, ... of an S^3 box
// (b in x-fastest order): the step's own coordinates are added with carries,
// so only the start takes integer divisions.
struct BoxWalk {
  int x, y, z, sx, sy, sz;
  __device__ __forceinline__ BoxWalk(int b, int step, int S)
      : x(b % S), y((b / S) % S), z(b / (S * S)), sx(step % S), sy((step / S) % S), sz(step / (S * S)) {}
  __device__ __forceinline__ void advance(int S) {
    x += sx;
    const int cx = x >= S ? 1 : 0;
    x -= cx * S;
    y += sy + cx;
    const int cy = y >= S ? 1 : 0;
    y -= cy * S;
    z += sz + cy;
  }
};

// box_node for the walker's current node.
__device__ __forceinline__ int box_node_at(const BoxWalk& w, const int (&lo)[3], const Geometry& g, int (&cc)[3]) {
  cc[0] = lo[0] + w.x;
  cc[1] = lo[1] + w.y;
  cc[2] = lo[2] + w.z;
  return wrap_coord(cc[0], g.nx) + g.nx * (wrap_coord(cc[1], g.ny) + g.ny * wrap_coord(cc[2], g.nz));
}

__device__ __forceinline__ void box_origin(const double* r, double R, int (&lo)[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) lo[a] = static_cast<int>(floor(r[a] - R)) - 1;
}

// The six sums of a particle's workgroup, combined in the fixed order above;
// valid in thread 0.
__device__ __forceinline__ void part_reduce(double (&acc)[6], double (&red)[4][6]) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 0; d < 6; ++d) acc[d] = wave_sum_xor(acc[d]);
  if (lane == 0)
#pragma unroll
    for (int d = 0; d < 6; ++d) red[wave][d] = acc[d];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int d = 0; d < 6; ++d) acc[d] = (red[0][d] + red[1][d]) + (red[2][d] + red[3][d]);
}

// Bounce-back at the particle's links, then force and torque from them,
// then leap-frog: v += F/m, omega += T/I, r += v.  One 256-thread workgroup
// per particle, on fnew just pushed by k1p_step (owner of step t).  For the
// link from fluid node x_f into the particle's node x_s = x_f + c_i, slot i
// of x_s holds f*_i(x_f); it becomes f_ibar(x_f, t+1) = f*_i(x_f) - W_i and
// the slot is cleared.  Every link of a node belongs to its owner, so each
// slot is touched by one workgroup.
//
// Only the shell R - 1.5 <= |d| <= R of the box can hold linked nodes of the
// particle (a node deeper in has all its neighbours inside).  The shell nodes
// are queued in LDS in box order, 256 at a time.  Each batch of 256 then
// runs in two phases, so that a thread waits for memory about three times
// per batch rather than once per chunk of directions:
//   1. thread l takes queue entry l: its owner, then the owners of its
//      neighbours outside the particle, all 18 loads at once, give the
//      node's links; the links are listed in LDS in queue order, directions
//      ascending (a prefix sum over the workgroup places them);
//   2. thread l takes list entries l, l + 256, ..., kLinkGroup at a time
//      with all their loads in flight together, and applies them.
// Both orders are fixed, so the float64 sums are repeatable.
//
// NC components: the populations of component k are planes k Q .. k Q + 18,
// its recorded densities rho_buf[k N ..]; each link is handled per
// component, component 0 first.  TILED: fnew is in the tile-major layout.
constexpr int kLinkGroup = 4;  // links a thread applies with their loads in flight together
template <int ST, int NC = 1, bool TILED = false>
__global__ void __launch_bounds__(kPartThreads) kp_force_move(store_t<ST>* __restrict__ fnew,
                                                              const int* __restrict__ owner,
                                                              const double* __restrict__ rho_buf, PartState ps,
                                                              Geometry g, StepCoeffs c) {
  using real = real_t<ST>;
  __shared__ double red[4][6];
  __shared__ int queue[2 * kPartThreads];
  __shared__ int wave_count[kPartThreads / 64];
  __shared__ int node_n[kPartThreads], node_x[kPartThreads], node_y[kPartThreads], node_z[kPartThreads];
  __shared__ int link_list[kPartThreads * (Q - 1)];  // (queue slot) * 32 + i
  const int p = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const PartRegs q = part_regs(ps, p);
  int lo[3];
  box_origin(q.r, ps.radius, lo);
  const int S = ps.box, nbox = S * S * S;
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};

  // exclusive prefix sum of v over the workgroup (thread order); total in `total`
  auto block_scan = [&](int v, int& total) -> int {
    int incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int u = __shfl_up(incl, d, 64);
      if (lane >= d) incl += u;
    }
    if (lane == 63) wave_count[wave] = incl;
    __syncthreads();
    int base = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < kPartThreads / 64; ++w) {
      base += w < wave ? wave_count[w] : 0;
      total += wave_count[w];
    }
    __syncthreads();  // wave_count is reused by the caller
    return base + incl - v;
  };

  // Phase 1 for the first `cnt` queue entries: list their links.  A
  // neighbour x_s - c_i inside this particle (the owner map's own test, on
  // the same unwrapped coordinates, so the same decision) is solid; the
  // others load their owner, and a fluid one makes a link.
  auto list_links = [&](int cnt) -> int {
    uint32_t mask = 0;
    const int t = threadIdx.x;
    if (t < cnt) {
      int cc[3];
      const int n = box_node(queue[t], lo, S, g, cc);
      if (owner[n] == p) {
        const int xs = wrap_coord(cc[0], g.nx), ys = wrap_coord(cc[1], g.ny), zs = wrap_coord(cc[2], g.nz);
        node_n[t] = n;
        node_x[t] = xs;
        node_y[t] = ys;
        node_z[t] = zs;
        int of[Q];
#pragma unroll
        for (int i = 1; i < Q; ++i) {
          const double ex = double(cc[0] - CX[i]) - q.r[0], ey = double(cc[1] - CY[i]) - q.r[1],
                       ez = double(cc[2] - CZ[i]) - q.r[2];
          const bool outside = (ex * ex + ey * ey) + ez * ez > ps.r2;
          const int nf = wrap_step(xs - CX[i], g.nx) + g.nx * (wrap_step(ys - CY[i], g.ny) + g.ny * wrap_step(zs - CZ[i], g.nz));
          of[i] = outside ? owner[nf] : p;  // inside this particle: solid
        }
#pragma unroll
        for (int i = 1; i < Q; ++i)
          if (owner_fluid(of[i])) mask |= 1u << i;
      }
    }
    int total = 0;
    int at = block_scan(__popc(mask), total);
    while (mask != 0) {
      const int i = __ffs(mask) - 1;
      mask &= mask - 1;
      link_list[at++] = t * 32 + i;
    }
    __syncthreads();
    return total;
  };

  // Phase 2: apply links j, j + 256, ... of the list.
  auto apply_links = [&](int total) {
    for (int j0 = threadIdx.x; j0 < total; j0 += kLinkGroup * kPartThreads) {
      int n[kLinkGroup], nf[kLinkGroup], dir[kLinkGroup], xs[kLinkGroup], ys[kLinkGroup], zs[kLinkGroup];
      real pushed[kLinkGroup][NC];
      double rh[kLinkGroup][NC];
#pragma unroll
      for (int u = 0; u < kLinkGroup; ++u) {
        const int j = j0 + u * kPartThreads;
        dir[u] = 0;
        if (j < total) {
          const int e = link_list[j], s = e >> 5, i = e & 31;
          dir[u] = i;
          n[u] = node_n[s];
          xs[u] = node_x[s];
          ys[u] = node_y[s];
          zs[u] = node_z[s];
          nf[u] = wrap_step(xs[u] - cx_of(i), g.nx) +
                  g.nx * (wrap_step(ys[u] - cy_of(i), g.ny) + g.ny * wrap_step(zs[u] - cz_of(i), g.nz));
#pragma unroll
          for (int kc = 0; kc < NC; ++kc) {
            pushed[u][kc] = decode_dir<ST>(fnew[pop_index<TILED>(kc * Q + i, n[u], xs[u], ys[u], zs[u], g)]);
            rh[u][kc] = rho_buf[(long long)kc * g.N + nf[u]];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < kLinkGroup; ++u) {
        const int i = dir[u];
        if (i == 0) continue;
        const int xf = wrap_step(xs[u] - cx_of(i), g.nx), yf = wrap_step(ys[u] - cy_of(i), g.ny),
                  zf = wrap_step(zs[u] - cz_of(i), g.nz);
#pragma unroll
        for (int kc = 0; kc < NC; ++kc) {
          double rb[3];
          const double W = wall_term(i, xf, yf, zf, rh[u][kc], q, g, rb);
          const store_t<ST> back = encode_dir<ST>(pushed[u][kc] - static_cast<real>(W));  // w_opp(i) = w_i
          fnew[pop_index<TILED>(kc * Q + opp_of(i), nf[u], xf, yf, zf, g)] = back;
          fnew[pop_index<TILED>(kc * Q + i, n[u], xs[u], ys[u], zs[u], g)] = store_t<ST>(0);
          const double gv = static_cast<double>(decode_dir<ST>(back));
          const double t = (gv + gv) + W;
          const double F[3] = {cx_of(i) == 0 ? 0.0 : (cx_of(i) > 0 ? t : -t), cy_of(i) == 0 ? 0.0 : (cy_of(i) > 0 ? t : -t),
                               cz_of(i) == 0 ? 0.0 : (cz_of(i) > 0 ? t : -t)};
          acc[0] = acc[0] + F[0];
          acc[1] = acc[1] + F[1];
          acc[2] = acc[2] + F[2];
          acc[3] = acc[3] + (rb[1] * F[2] - rb[2] * F[1]);
          acc[4] = acc[4] + (rb[2] * F[0] - rb[0] * F[2]);
          acc[5] = acc[5] + (rb[0] * F[1] - rb[1] * F[0]);
        }
      }
    }
    __syncthreads();  // the node table and the list are refilled by the next batch
  };

  int pending = 0;  // queued shell nodes, the same in every thread (below 256 between rounds)
  BoxWalk bw(threadIdx.x, kPartThreads, S);
  for (int b0 = 0; b0 < nbox; b0 += kPartThreads, bw.advance(S)) {
    const int b = b0 + threadIdx.x;
    bool shell = false;
    if (b < nbox) {
      int cc[3];
      box_node_at(bw, lo, g, cc);
      const double dx = double(cc[0]) - q.r[0], dy = double(cc[1]) - q.r[1], dz = double(cc[2]) - q.r[2];
      const double d2 = (dx * dx + dy * dy) + dz * dz;
      shell = d2 <= ps.r2 && d2 >= ps.inner2;
    }
    const unsigned long long m = __ballot(shell);
    if (lane == 0) wave_count[wave] = __popcll(m);
    __syncthreads();
    int slot = pending, total = 0;
#pragma unroll
    for (int w = 0; w < kPartThreads / 64; ++w) {
      slot += w < wave ? wave_count[w] : 0;
      total += wave_count[w];
    }
    if (shell) queue[slot + __popcll(m & ((1ull << lane) - 1ull))] = b;  // slot + rank < 2 * 256
    pending += total;
    __syncthreads();
    if (pending >= kPartThreads) {
      apply_links(list_links(kPartThreads));
      if (threadIdx.x < pending - kPartThreads) queue[threadIdx.x] = queue[kPartThreads + threadIdx.x];
      pending -= kPartThreads;
      __syncthreads();
    }
  }
  if (pending > 0) apply_links(list_links(pending));
  part_reduce(acc, red);
  if (threadIdx.x == 0) {
    const double L[3] = {double(g.nx), double(g.ny), double(g.nz)};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      ps.force[3 * p + a] = acc[a];
      ps.torque[3 * p + a] = acc[3 + a];
      const double v = ps.vel[3 * p + a] + acc[a] / ps.mass;
      ps.vel[3 * p + a] = v;
      ps.omg[3 * p + a] = ps.omg[3 * p + a] + acc[3 + a] / ps.inertia;
      double r = ps.pos[3 * p + a] + v;
      if (r >= L[a]) r = r - L[a];
      if (r < 0.0) r = r + L[a];
      ps.pos[3 * p + a] = r;
    }
  }
}

__global__ void __launch_bounds__(kBlock) kp_owner_fill(int* __restrict__ owner, int N) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n < N) owner[n] = kOwnerFluid;
}

// owner[x] = min over particles containing x (kOwnerNear within R + 1.5).
// One workgroup per particle.
__global__ void __launch_bounds__(kBlock) kp_owner_scatter(int* __restrict__ owner, PartState ps, Geometry g) {
  const int p = blockIdx.x;
  const double* r = ps.pos + 3 * p;
  int lo[3];
  box_origin(r, ps.radius, lo);
  const int S = ps.box, nbox = S * S * S;
  BoxWalk bw(threadIdx.x, kBlock, S);
  for (int b = threadIdx.x; b < nbox; b += kBlock, bw.advance(S)) {
    int cc[3];
    const int n = box_node_at(bw, lo, g, cc);
    const double dx = double(cc[0]) - r[0], dy = double(cc[1]) - r[1], dz = double(cc[2]) - r[2];
    const double d2 = (dx * dx + dy * dy) + dz * dz;
    if (d2 <= ps.r2) atomicMin(owner + n, p);
    else if (d2 <= ps.near2) atomicMin(owner + n, kOwnerNear);
  }
}

// Covering and uncovering after the move; mask follows the new owner map.
// NC components, each handled in turn at a node, component 0 first.  TILED:
// f is in the tile-major layout.
template <int ST, int NC = 1, bool TILED = false>
__global__ void __launch_bounds__(kPartThreads) kp_remap(store_t<ST>* __restrict__ f, const int* __restrict__ owner_old,
                                                         const int* __restrict__ owner_new, uint8_t* __restrict__ mask,
                                                         PartState ps, Geometry g, StepCoeffs c) {
  using real = real_t<ST>;
  __shared__ double red[4][6];
  const int p = blockIdx.x;
  const double* r = ps.pos + 3 * p;
  int lo[3];
  box_origin(r, ps.radius, lo);
  const int S = ps.box, nbox = S * S * S;
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  BoxWalk bw(threadIdx.x, kPartThreads, S);
  for (int b = threadIdx.x; b < nbox; b += kPartThreads, bw.advance(S)) {
    int cc[3];
    const int n = box_node_at(bw, lo, g, cc);
    const bool covered = owner_new[n] == p && owner_fluid(owner_old[n]);
    const bool uncovered = owner_old[n] == p && owner_fluid(owner_new[n]);
    if (!covered && !uncovered) continue;
    const double d[3] = {double(cc[0]) - r[0], double(cc[1]) - r[1], double(cc[2]) - r[2]};
    const int wx = wrap_coord(cc[0], g.nx), wy = wrap_coord(cc[1], g.ny), wz = wrap_coord(cc[2], g.nz);
    mask[n] = covered ? 1 : 0;
#pragma unroll
    for (int kc = 0; kc < NC; ++kc) {
      real vals[Q];
      double sign;
      if (covered) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const long long at = pop_index<TILED>(kc * Q + i, n, wx, wy, wz, g);
          vals[i] = decode<ST>(f[at], c.shift[kc][i]);
          f[at] = store_t<ST>(0);
        }
        sign = 1.0;
      } else {
        const double* v = ps.vel + 3 * p;
        const double* w = ps.omg + 3 * p;
        const double ub[3] = {v[0] + (w[1] * d[2] - w[2] * d[1]), v[1] + (w[2] * d[0] - w[0] * d[2]),
                              v[2] + (w[0] * d[1] - w[1] * d[0])};
        const real ux = static_cast<real>(ub[0]), uy = static_cast<real>(ub[1]), uz = static_cast<real>(ub[2]);
        const real rho0 = static_cast<real>(ps.rho0[kc]);
        const real t15 = real(1.5) * ((ux * ux + uy * uy) + uz * uz);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const real cu = cdot<real>(i, ux, uy, uz);
          const real feq = (weight<real>(i) * rho0) * (((real(1) + real(3) * cu) + real(4.5) * cu * cu) - t15);
          const store_t<ST> sv = encode<ST>(feq, c.shift[kc][i]);
          f[pop_index<TILED>(kc * Q + i, n, wx, wy, wz, g)] = sv;
          vals[i] = decode<ST>(sv, c.shift[kc][i]);  // the stored value, so that the exchange is exact
        }
        sign = -1.0;
      }
      const double m[3] = {sign * static_cast<double>(lattice_sum<0, 0, real>(vals)),
                           sign * static_cast<double>(lattice_sum<1, 0, real>(vals)),
                           sign * static_cast<double>(lattice_sum<2, 0, real>(vals))};
      acc[0] = acc[0] + m[0];
      acc[1] = acc[1] + m[1];
      acc[2] = acc[2] + m[2];
      acc[3] = acc[3] + (d[1] * m[2] - d[2] * m[1]);
      acc[4] = acc[4] + (d[2] * m[0] - d[0] * m[2]);
      acc[5] = acc[5] + (d[0] * m[1] - d[1] * m[0]);
    }
  }
  part_reduce(acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      ps.vel[3 * p + a] = ps.vel[3 * p + a] + acc[a] / ps.mass;
      ps.omg[3 * p + a] = ps.omg[3 * p + a] + acc[3 + a] / ps.inertia;
    }
  }
}

// Initial owner-based state: zero the populations of solid nodes (NC
// components), mask = owner != fluid.
template <int ST, int NC = 1>
__global__ void __launch_bounds__(kBlock) kp_apply_owner(store_t<ST>* __restrict__ f, const int* __restrict__ owner,
                                                         uint8_t* __restrict__ mask, Geometry g) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= g.N) return;
  const bool solid = !owner_fluid(owner[n]);
  mask[n] = solid ? 1 : 0;
  if (solid)
#pragma unroll
    for (int i = 0; i < NC * Q; ++i) f[(long long)i * g.Npad + n] = store_t<ST>(0);
}

// Particles removed: their nodes turn to fluid at rest, f^k_i = w_i rho0_k.
template <int ST, int NC = 1>
__global__ void __launch_bounds__(kBlock) kp_release(store_t<ST>* __restrict__ f, uint8_t* __restrict__ mask,
                                                     double rho0a, double rho0b, Geometry g, StepCoeffs c) {
  using real = real_t<ST>;
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= g.N || !mask[n]) return;
  mask[n] = 0;
#pragma unroll
  for (int kc = 0; kc < NC; ++kc)
#pragma unroll
    for (int i = 0; i < Q; ++i)
      f[(long long)(kc * Q + i) * g.Npad + n] =
          encode<ST>(weight<real>(i) * static_cast<real>(kc == 0 ? rho0a : rho0b), c.shift[kc][i]);
}

}  // namespace lbd
