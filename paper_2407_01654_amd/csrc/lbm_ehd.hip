// C-ABI library for the coupled two-phase EHD lattice Boltzmann step on gfx950.
// Kernels: the round kernel (per tile, its instance's main pass of g, l, f or
// one potential iteration of h), the per-instance finalize (ordered FP64
// reductions, stop test, next phase), the start of a stepping call,
// initialisation and field extraction.  Rounds run in hipGraph-captured
// chunks steered by device-side state.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <chrono>
#include <vector>

#include "lbm_ehd.h"
#include "lbm_ehd_device.hpp"

using namespace lbm;

namespace {


// ---------------------------------------------------------------------------
// per-instance inner-loop bookkeeping (shared by the host-steered and the
// persistent paths)
// ---------------------------------------------------------------------------
struct LoopState {
  int active, k, target, hpar, rpos, rpar, reref;
};

__device__ inline LoopState loop_begin(const InstDyn& d, const InstConst& C, const int* replay_row,
                                       bool presolve) {
  LoopState L;
  L.active = (C.enable & EN_POT) ? 1 : 0;
  L.k = 0;
  L.hpar = d.h_par;
  L.rpos = d.replay_pos;
  L.rpar = d.ref_par;
  L.reref = presolve ? 0 : 1;  // the first iteration of a step moves h to the new reference
  if (presolve) {
    L.target = C.presolve_iters;
  } else if (L.rpos < d.replay_n) {
    L.target = replay_row[L.rpos];
    L.rpos++;
  } else {
    L.target = 0;
  }
  return L;
}

// Long inner loops move h to a fresh reference every REREF_EVERY iterations:
// iteration k captures psi^(k) into the spare reference plane, iteration k+1
// re-encodes h relative to it.
constexpr int REREF_EVERY = 64;
__device__ inline int capture_of(const LoopState& L) {
  return (!L.reref && (L.k + 1) % REREF_EVERY == 0) ? 1 : 0;
}

// Applies the stop test of Algorithm 1 step 3 after one iteration.  num:
// sum of the squared successive changes of psi, den: sum of psi^2, fl: sum of
// the squared changes of psi that rounding the stored h to 16 bits alone
// makes (0 with FP32 storage).  Besides r < tol the loop also ends, without
// forced counts, once num is within 4 fl: the successive change is then no
// larger than twice the change rounding alone produces, and further
// iterations only resample that rounding.  Such an end sets bit 2 (value 4)
// of status_bits.
__device__ inline bool loop_iterate(LoopState& L, const InstConst& C, double num, double den, double fl,
                                    double& r, int& status_bits) {
  const int captured = capture_of(L);
  L.k += 1;
  L.hpar ^= 1;
  if (L.reref) {
    L.rpar ^= 1;
    L.reref = 0;
  } else if (captured) {
    L.reref = 1;
  }
  const double floor_den = 1e-300 * (double)C.nx * (double)C.ny;
  r = sqrt(num / (den > floor_den ? den : floor_den));
  bool stop;
  if (!isfinite(r)) {
    status_bits |= 2;
    stop = true;
  } else if (L.target > 0) {
    stop = L.k >= L.target;
  } else {
    const bool at_floor = !(r < C.tol) && num <= 4.0 * fl;
    stop = r < C.tol || at_floor || L.k >= C.max_iter;
    if (at_floor) status_bits |= 4;
    else if (!(r < C.tol) && L.k >= C.max_iter) status_bits |= 1;
  }
  if (stop) L.active = 0;
  return stop;
}

// writes the finished loop into the instance record
__device__ inline void loop_commit(InstDyn& d, const LoopState& L, double r, int status_bits,
                                   int* khist_row, bool presolve) {
  d.h_par = L.hpar;
  d.ref_par = L.rpar;
  d.reref = L.reref;
  d.k = L.k;
  d.active = 0;
  d.replay_pos = L.rpos;
  d.last_r = r;
  d.status |= status_bits;
  if (presolve) {
    d.presolve_k = L.k;
    khist_row[0] = L.k;
  } else {
    d.steps += 1;
    d.total_iters += L.k;
    khist_row[d.steps % HIST] = L.k;
  }
}

// deterministic sum of per-tile partials [b, e) of two arrays.  Each thread
// adds its partials in a fixed order; the unrolling only lets the loads of 16
// of them be in flight together (a single instance of 8192 tiles gives each
// thread 32 partials, whose loads would otherwise form a chain of round trips)
__device__ inline double3 sum_parts3(const double2* part, const double* part2, int b, int e, double* red) {
  double a = 0.0, c = 0.0, f = 0.0;
#pragma unroll 16
  for (int j = b + (int)threadIdx.x; j < e; j += blockDim.x) {
    const double2 v = part[j];
    a += v.x;
    c += v.y;
    f += part2[j];
  }
  return block_sum3(a, c, f, red);
}

// deterministic sum of per-tile partials [b, e)
__device__ inline double2 sum_parts(const double2* part, int b, int e, double* red) {
  double a = 0.0, c = 0.0;
#pragma unroll 16
  for (int j = b + (int)threadIdx.x; j < e; j += blockDim.x) {
    const double2 v = part[j];
    a += v.x;
    c += v.y;
  }
  return block_sum2(a, c, red);
}

// ---------------------------------------------------------------------------
// stepping: rounds.  In one round every tile performs its own instance's
// current phase (main pass or one inner iteration), then one workgroup per
// instance reduces the instance's partial sums in a fixed order, applies the
// stop test and moves the instance to its next phase.  Instances advance
// independently (an instance iterating its potential does not hold up the
// others), and kernel boundaries order the data between phases: no grid-wide
// synchronisation inside a kernel.
// ---------------------------------------------------------------------------
// an instance whose state turned non-finite (status flag 2) is retired: its
// tiles are skipped from then on and the other instances carry on
__device__ __forceinline__ bool inst_active(const InstDyn& d) {
  if (d.status & 2) return false;
  return d.presolve ? true : d.s_done < d.n_target;
}

// start of a stepping call: n_target outer steps, or the initial potential
// solve; counters[0] = instances of the round path with nothing to do;
// counters[1] / [2] count the main passes / inner iterations the round path
// performs during the call
__global__ void __launch_bounds__(256) k_begin(Ctx c, int n_target, int presolve) {
  __shared__ int s_cnt;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  int idle = 0;
  for (int i = threadIdx.x; i < c.n_inst; i += blockDim.x) {
    InstDyn& d = c.dyn[i];
    const InstConst& C = c.ic[i];
    d.s_done = 0;
    d.n_target = n_target;
    if (presolve) {
      const LoopState L = loop_begin(d, C, c.replay + (long long)i * HIST, true);
      d.presolve = L.active;
      d.phase = 1;
      d.k = 0;
      d.target = L.target;
      d.reref = 0;
      if (!L.active) {
        d.presolve_k = 0;
        c.khist[(long long)i * HIST] = 0;
        d.phase = 0;
      }
    }
    // staggered instances sit out the first round of a stepping call, so that
    // their main passes fall in the same rounds as the others' inner
    // iterations
    if (!presolve && C.stagger && !C.solo && inst_active(d) && d.phase == 0) d.phase = 2;
    if (!inst_active(d) && !C.solo) ++idle;
  }
  atomicAdd(&s_cnt, idle);
  __syncthreads();
  if (threadIdx.x == 0) {
    c.counters[0] = s_cnt;
    c.counters[1] = 0;
    c.counters[2] = 0;
  }
}

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on
// XCD b mod 8), each with its own L2.  Workgroup b takes block xcd_tile(b) of
// the work list, so that every XCD takes one contiguous range of it:
// neighbouring strips of a band, and neighbouring bands, then share an L2 and
// the lines that straddle a strip edge are fetched once.
__device__ __forceinline__ int xcd_tile(int b, int nt) {
  const int q = nt >> 3, r = nt & 7, xcd = b & 7, j = b >> 3;
  return (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + j;
}

// One wave advances tile ti by its instance's current phase (main pass or one
// inner iteration) and writes the tile's partial sums (wave reductions).
// The tile and the instance record are the same for the whole wave; saying
// so keeps every plane offset derived from them in scalar registers.
template <class S>
__device__ __forceinline__ void tile_work(const Ctx& c, int ti) {
  const int4 tq = c.tiles[ti];
  const int inst = __builtin_amdgcn_readfirstlane(tq.x), x0 = __builtin_amdgcn_readfirstlane(tq.y);
  const int y0 = __builtin_amdgcn_readfirstlane(tq.z), y1 = __builtin_amdgcn_readfirstlane(tq.w);
  const InstDyn& D = c.dyn[inst];
  if (!inst_active(D)) return;
  const InstConst C = c.ic[inst];
  const int bin = __builtin_amdgcn_readfirstlane(D.bin);
  const int ref_par = __builtin_amdgcn_readfirstlane(D.ref_par);
  const bool lead = (threadIdx.x & 63) == 0;
  const int phase = __builtin_amdgcn_readfirstlane(D.phase);
  if (phase == 2) return;
  if (phase == 0) {
    double aphi = 0.0, aq = 0.0;
    main_tile<S>(c, C, x0, y0, y1, bin, ref_par ^ 1, aphi, aq);
    aphi = wave_sum(aphi);
    aq = wave_sum(aq);
    if (lead) c.part_main[ti] = make_double2(aphi, aq);
  } else {
    LoopState L;
    L.k = __builtin_amdgcn_readfirstlane(D.k);
    L.reref = __builtin_amdgcn_readfirstlane(D.reref);
    const int rdec = ref_par, renc = rdec ^ (L.reref & 1);  // integer form: stays scalar
    // phi^n: written by this step's main pass into the other phi plane (both
    // planes hold phi^0 during the initial solve)
    const int phip = __builtin_amdgcn_readfirstlane(D.presolve) ? bin : bin ^ 1;
    const int hpar = __builtin_amdgcn_readfirstlane(D.h_par);
    double num = 0.0, den = 0.0, fl = 0.0;
    pot_tile<S>(c, C, x0, y0, y1, hpar, phip, rdec, renc, capture_of(L), num, den, fl);
    num = wave_sum(num);
    den = wave_sum(den);
    fl = wave_sum(fl);
    if (lead) {
      c.part_pot[ti] = make_double2(num, den);
      c.part_floor[ti] = fl;
    }
  }
}

// One round over the round path's part of the work list (every instance that
// is not solo).  A workgroup holds blockDim.x / 64 waves and each wave
// advances one tile on its own (adjacent strips share the compute unit and
// its caches; no barrier, no LDS).  Register budget: 4 waves per SIMD (128
// VGPRs) holds both passes without spills; at 5 waves the main pass spilled
// 10-23 VGPRs and ran 10-17 % slower on the sweep, while the inner iteration
// was 2-11 % faster.
template <class S>
__global__ void __launch_bounds__(256, 4) k_round(Ctx c) {
  const int wpb = (int)(blockDim.x >> 6);
  const int nb = (c.n_ns_tiles + wpb - 1) / wpb;
  const int ti = __builtin_amdgcn_readfirstlane(xcd_tile((int)blockIdx.x, nb) * wpb + (int)(threadIdx.x >> 6));
  if (ti >= c.n_ns_tiles) return;
  tile_work<S>(c, ti);
}

// Reduction, stop test and next phase of instance i after a pass over its
// tiles, by a workgroup of FIN_THREADS threads (the finalize kernel's, or the
// instance's own in k_solo: the partials are summed in the same order either
// way).  Thread 0 updates the instance record.  The round path's instances
// count their passes and their end in counters[1], [2] and [0]; solo ones
// touch no counter.
constexpr int FIN_THREADS = 256;
__device__ __forceinline__ void finalize_instance(const Ctx& c, int i, double* red, bool solo) {
  InstDyn& D = c.dyn[i];
  if (!inst_active(D)) return;
  const InstConst& C = c.ic[i];
  int* khist_row = c.khist + (long long)i * HIST;
  bool finished = false;
  const int phase = D.phase;
  if (phase == 2) {  // the staggered start's idle round is over
    if (threadIdx.x == 0) D.phase = 0;
    return;
  }
  if (!solo && threadIdx.x == 0) atomicAdd(&c.counters[phase == 0 ? 1 : 2], 1);
  if (phase == 0) {
    const double2 sm = sum_parts(c.part_main, C.tile_begin, C.tile_end, red);
    if (threadIdx.x == 0) {
      D.sum_phi = sm.x;
      D.sum_q = sm.y;
      const LoopState L = loop_begin(D, C, c.replay + (long long)i * HIST, false);
      if (!isfinite(sm.x) || !isfinite(sm.y)) {
        D.status |= 2;  // retired; it no longer holds up the call
        finished = true;
      } else if (L.active) {
        D.phase = 1;
        D.k = 0;
        D.target = L.target;
        D.replay_pos = L.rpos;
        D.reref = L.reref;
      } else {
        D.steps += 1;
        khist_row[D.steps % HIST] = 0;
        D.bin ^= 1;
        D.s_done += 1;
        finished = D.s_done >= D.n_target;
      }
    }
  } else {
    double3 sp = sum_parts3(c.part_pot, c.part_floor, C.tile_begin, C.tile_end, red);
    if (C.pot_stop) {  // the Poisson residual of the new psi replaces the successive change
      const double2 sr = sum_parts(c.part_res, C.tile_begin, C.tile_end, red);
      sp = make_double3(sr.x, sr.y, 0.0);
    }
    if (threadIdx.x == 0) {
      LoopState L;
      L.active = 1;
      L.k = D.k;
      L.target = D.target;
      L.hpar = D.h_par;
      L.rpos = D.replay_pos;
      L.rpar = D.ref_par;
      L.reref = D.reref;
      double r;
      int bits = 0;
      const bool stop = loop_iterate(L, C, sp.x, sp.y, sp.z, r, bits);
      D.k = L.k;
      D.h_par = L.hpar;
      D.ref_par = L.rpar;
      D.reref = L.reref;
      D.last_r = r;
      if (C.pot_stop) D.last_res = r;
      if (stop) {
        const bool pre = D.presolve != 0;
        if (bits & 4) D.floor_stops += 1;
        loop_commit(D, L, r, bits & 3, khist_row, pre);
        D.phase = 0;
        if (pre || (bits & 2)) {  // end of the initial solve, or retired
          D.presolve = 0;
          finished = true;
        } else {
          D.bin ^= 1;
          D.s_done += 1;
          finished = D.s_done >= D.n_target;
        }
      }
    }
  }
  if (finished && !solo) atomicAdd(&c.counters[0], 1);
}

// one workgroup per instance of the round path: reduction, stop test, next phase
__global__ void __launch_bounds__(FIN_THREADS) k_finalize(Ctx c) {
  __shared__ double red[48];
  if (c.ic[blockIdx.x].solo) return;
  finalize_instance(c, (int)blockIdx.x, red, false);
}

// One workgroup per solo instance (small lattices) advances it through the
// whole stepping call on its own, beside the rounds of the other instances
// on a second stream: its waves share the instance's tiles, and after every
// pass the workgroup reduces the partial sums and takes the stop decision
// itself, so that an inner iteration costs a workgroup barrier instead of a
// round of the device, and an instance with long inner loops no longer sets
// the number of rounds of the call.  The tiles, their arithmetic and the
// order of every sum are those of the round path: the results are the same
// bit for bit.  Workgroup barriers order the passes (the waves of a
// workgroup share one compute unit and its L1).  The register budget is the
// kernel's own (one workgroup of 4 waves per compute unit at most).
template <class S>
__global__ void __launch_bounds__(FIN_THREADS) k_solo(Ctx c) {
  __shared__ double red[48];
  const int inst = c.solo_list[blockIdx.x];
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int t0 = c.ic[inst].tile_begin, t1 = c.ic[inst].tile_end;
  while (inst_active(c.dyn[inst])) {
    for (int ti = t0 + wave; ti < t1; ti += FIN_THREADS / WAVE) tile_work<S>(c, ti);
    __syncthreads();
    finalize_instance(c, inst, red, true);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Poisson residual of Eq. (52) in the flux form of the lattice, per tile: for
// every node r = sum_i (2 w_i / c_s^2) eps_i (psi(x + c_i) - psi(x)) + q with
// eps_i the harmonic mean of eps(phi) at both ends (the node's own across an
// electrode, where psi is the ghost 2 psi_w - psi(x + c_i - c_iy e_y)), and s
// the sum of the magnitudes of its terms; the tile's sums of r^2 and s^2 in
// FP64.  The psi plane holds psi - psi_lin, so a difference along c_i adds
// c_iy glin, and the ghost's deviation is minus that of its mirror node.
// only >= 0: instance `only` between steps (phi^n, q^n of its last main pass);
// only < 0: the instances iterating with the residual stop test, after the
// round's inner iteration (psi just gathered).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(WAVE) k_residual(Ctx c, int only) {
  const int ti = (int)blockIdx.x;
  if (ti >= c.n_tiles) return;
  const int4 tq = c.tiles[ti];
  const int inst = tq.x;
  const InstDyn& D = c.dyn[inst];
  const InstConst& C = c.ic[inst];
  int phip;
  if (only >= 0) {
    if (inst != only) return;
    phip = D.bin;
  } else {
    if (!C.pot_stop || !inst_active(D) || D.phase != 1) return;
    phip = D.presolve ? D.bin : D.bin ^ 1;
  }
  const float* pool = c.fpool + C.off_f;
  auto at = [&](int pid, int xx, int yy) {
    return pool[(long long)yy * C.ldx + col_slot(xx) + (long long)pid * C.plane];
  };
  auto eps_of = [&](float ph) { return (double)C.eps_v + (double)ph * ph * (2.0 * ph - 3.0) * (double)C.deps; };
  const int x = tq.y + (int)threadIdx.x;
  double a = 0.0, b = 0.0;
  if (x < min(tq.y + STRIP, C.nx)) {
    for (int y = tq.z; y < tq.w; ++y) {
      const double e0 = eps_of(at(AUX_PHI0 + phip, x, y));
      const double p0 = at(AUX_PSI, x, y), q = at(AUX_Q0 + phip, x, y);
      double r = q, sa = fabs(q);
      for (int i = 1; i < 9; ++i) {
        const int xs = wrapi(x + CX[i], C.nx), ys = y + CY[i];
        double ei, pn;
        if (C.walls && (ys < 0 || ys >= C.ny)) {
          ei = e0;
          pn = -(double)at(AUX_PSI, xs, y);
        } else {
          const int yw = wrapi(ys, C.ny);
          const double e1 = eps_of(at(AUX_PHI0 + phip, xs, yw));
          ei = 2.0 * e0 * e1 / (e0 + e1);
          pn = at(AUX_PSI, xs, yw);
        }
        const double t = 2.0 * (double)W9[i] * 3.0 * ei * (pn - p0 + (double)CY[i] * (double)C.glin);
        r += t;
        sa += fabs(t);
      }
      a += r * r;
      b += sa * sa;
    }
  }
  a = wave_sum(a);
  b = wave_sum(b);
  if (threadIdx.x == 0) c.part_res[ti] = make_double2(a, b);
}

// ---------------------------------------------------------------------------
// initialisation and field extraction (one node per thread, not hot)
// ---------------------------------------------------------------------------
struct NodeIdx {
  int x, y;
  long long idx;
};

__device__ inline bool node_of(const InstConst& C, NodeIdx& n) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (long long)C.nx * C.ny) return false;
  n.y = (int)(g / C.nx);
  n.x = (int)(g % C.nx);
  n.idx = (long long)n.y * C.ldx + col_slot(n.x);
  return true;
}

// value of a plane at (x, y) with wall ghosts: kind 0 order parameter, 1
// potential; padded: pool plane (strip slots) or compact [ny][nx] plane
__device__ inline float at_ghost(const InstConst& C, const float* pl, int x, int y, int kind, bool padded) {
  x = wrapi(x, C.nx);
  const long long ld = padded ? C.ldx : C.nx;
  const int xs = padded ? col_slot(x) : x;
  if (!C.walls) return pl[(long long)wrapi(y, C.ny) * ld + xs];
  if (y < 0) {
    const float a = pl[xs], b = pl[ld + xs];
    return kind == 0 ? phi_ghost(a, b, C.wet_b) : -a;
  }
  if (y >= C.ny) {
    const float a = pl[(long long)(C.ny - 1) * ld + xs], b = pl[(long long)(C.ny - 2) * ld + xs];
    return kind == 0 ? phi_ghost(a, b, C.wet_t) : -a;
  }
  return pl[(long long)y * ld + xs];
}

__device__ inline void stencil_at(const InstConst& C, const float* pl, int x, int y, int kind, bool padded,
                                  float& gx, float& gy, float& lap) {
  const float c0 = at_ghost(C, pl, x, y, kind, padded);
  gx = gy = lap = 0.f;
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const float v = at_ghost(C, pl, x + CX[i], y + CY[i], kind, padded);
    gx += W9[i] * CX[i] * v;
    gy += W9[i] * CY[i] * v;
    lap += 2.f * W9[i] * (v - c0);
  }
  gx *= INV_CS2;
  gy *= INV_CS2;
  lap *= INV_CS2;
}

// Writes node-level pre-collision populations pop[] of (x, y) into the
// post-collision buffer at the places the next pull reads them from.
// off(j, x, y): storage offset of direction j at the storing node (x, y).
template <class S, class Off>
__device__ inline void place_prepulled(const PopView<S>& v, const InstConst& C, int set, int x, int y,
                                       const float pop[9], bool anti, Off off) {
  for (int i = 0; i < 9; ++i) {
    const int ys = y - CY[i];
    if (C.walls && (ys < 0 || ys >= C.ny)) {
      const float pw = ys < 0 ? C.psi_b : C.psi_t;
      const float val = anti ? 2.f * W9[i] * pw - pop[i] : pop[i];
      v.put(OPP[i], (unsigned)(y * C.ldx + col_slot(x)), val, set, C, off(OPP[i], x, y));
    } else {
      const int xs = wrapi(x - CX[i], C.nx), yw = wrapi(ys, C.ny);
      v.put(i, (unsigned)(yw * C.ldx + col_slot(xs)), pop[i], set, C, off(i, xs, yw));
    }
  }
}

// Initial potential: the linear profile between the electrodes (zero when y is
// periodic).  The psi and reference planes hold deviations from that profile,
// so they start at zero; h starts at its equilibrium, stored relative to it.
template <class S>
__global__ void k_init_h(Ctx c, int inst) {
  const InstConst C = c.ic[inst];
  NodeIdx n;
  if (!node_of(C, n)) return;
  c.fpool[C.off_f + (long long)AUX_PSI * C.plane + n.idx] = 0.f;
  c.fpool[C.off_f + (long long)AUX_REF0 * C.plane + n.idx] = 0.f;
  const PopView<S> hv(make_pools<S>(c, C), 0, SET_H);
  // h_i^eq(psi_lin(y)) pulled into (x, y) from (x, y) - c_i, minus k_i psi_lin
  // of the storing node: k_i c_iy glin; across a wall the anti-bounce-back
  // value 2 w_i psi_wall - h_i stored as direction opp(i) of (x, y)
  for (int i = 0; i < 9; ++i) {
    const int ys = n.y - CY[i];
    if (C.walls && (ys < 0 || ys >= C.ny)) {
      const float half = ys < 0 ? -0.5f * C.glin : 0.5f * C.glin;  // psi_wall - psi_lin(y)
      hv.put(OPP[i], (unsigned)n.idx, 2.f * W9[i] * half, SET_H, C);
    } else {
      const int xs = wrapi(n.x - CX[i], C.nx), yw = wrapi(ys, C.ny);
      hv.put(i, (unsigned)(yw * C.ldx + col_slot(xs)), KH[i] * (float)CY[i] * C.glin, SET_H, C);
    }
  }
}

// init[0..N): u_x, [N..2N): u_y (only if has_u), [2N..3N): phi0 - fl32(phi0); compact [ny][nx]
template <class S>
__global__ void k_init_pops(Ctx c, int inst, const float* init, int has_u) {
  const InstConst C = c.ic[inst];
  NodeIdx n;
  if (!node_of(C, n)) return;
  float* aux = c.fpool + C.off_f;
  const float* phi_pl = aux + (long long)AUX_PHI0 * C.plane;
  const float* psi_pl = aux + (long long)AUX_PSI * C.plane;
  float gphx, gphy, lphi, gpsx, gpsy, lpsi;
  stencil_at(C, phi_pl, n.x, n.y, 0, true, gphx, gphy, lphi);
  stencil_at(C, psi_pl, n.x, n.y, 1, true, gpsx, gpsy, lpsi);
  const float phi = phi_pl[n.idx];
  const float* q_pl = aux + (long long)AUX_Q0 * C.plane;
  const float q = q_pl[n.idx];
  const long long N = (long long)C.nx * C.ny, cidx = (long long)n.y * C.nx + n.x;
  float ux = 0.f, uy = 0.f;
  if (has_u && (C.enable & EN_HYDRO)) {
    ux = init[cidx];
    uy = init[N + cidx];
  }
  const float resid = init[2 * N + cidx];
  const float Ex = -gpsx, Ey = -gpsy - C.glin;  // psi plane holds psi - psi_lin
  const float deps = 6.f * phi * (phi - 1.f) * C.deps;
  const float mu_c = C.beta4 * phi * (phi - 0.5f) * (phi - 1.f) - C.kappa * lphi - 0.5f * deps * (Ex * Ex + Ey * Ey);
  const float rho = C.rho_v + phi * C.drho;
  const float uu = ux * ux + uy * uy;
  // implicit charge closure: sum l^0 = q0 - R^0 / 2 makes Eq. (66) return q0
  float R0 = 0.f;
  if (C.q_impl) {
    const float eps = C.eps_v + phi * phi * (2.f * phi - 3.f) * C.deps, sig = C.sig_v + phi * C.dsig;
    const float gE = gphx * Ex + gphy * Ey;
    R0 = -sig * q / eps + (sig / eps) * deps * gE - C.dsig * gE;
  }
  float g[9], l[9], f[9];
  for (int i = 0; i < 9; ++i) {
    const float cu = CX[i] * ux + CY[i] * uy;
    // g_0 is stored as its deviation from the phi plane (fl32(phi0))
    g[i] = i == 0 ? resid - (1.f - W9[0]) * mu_c : W9[i] * mu_c;
    l[i] = W9[i] * (q * (1.f + cu * INV_CS2) - 0.5f * R0);
    f[i] = rho * W9[i] * (cu * INV_CS2 + cu * cu * (0.5f * INV_CS2 * INV_CS2) - uu * (0.5f * INV_CS2));
  }
  auto none = [](int, int, int) { return 0.f; };
  // l_i relative to w_i times the charge of the storing node (both q planes hold q0)
  auto lref = [&](int j, int xx, int yy) {
    return S::kChargeRef ? W9[j] * q_pl[(long long)yy * C.ldx + col_slot(xx)] : 0.f;
  };
  const Pools P = make_pools<S>(c, C);
  for (int b = 0; b < 2; ++b) {
    place_prepulled<S>(PopView<S>(P, b, SET_G), C, SET_G, n.x, n.y, g, false, none);
    place_prepulled<S>(PopView<S>(P, b, SET_L), C, SET_L, n.x, n.y, l, false, lref);
    place_prepulled<S>(PopView<S>(P, b, SET_F), C, SET_F, n.x, n.y, f, false, none);
  }
  aux[(long long)AUX_FX * C.plane + n.idx] = 0.f;
  aux[(long long)AUX_FY * C.plane + n.idx] = 0.f;
  aux[(long long)AUX_R * C.plane + n.idx] = 0.f;
  aux[(long long)AUX_GAM * C.plane + n.idx] = ux * gphx + uy * gphy;
  aux[(long long)AUX_JX * C.plane + n.idx] = q * ux;
  aux[(long long)AUX_JY * C.plane + n.idx] = q * uy;
}

// scatter compact host-order planes into the padded aux planes
__global__ void k_put_plane(float* dst, const float* src, int nx, int ny, int ldx) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (long long)nx * ny) return;
  const int y = (int)(g / nx), x = (int)(g % nx);
  dst[(long long)y * ldx + col_slot(x)] = src[g];
}

// level-n order parameter into scratch plane 0 (compact)
template <class S>
__global__ void k_fields_phi(Ctx c, int inst, float* scr) {
  const InstConst C = c.ic[inst];
  const int bin = c.dyn[inst].bin;
  NodeIdx n;
  if (!node_of(C, n)) return;
  float g[9];
  const float hi = c.fpool[C.off_f + (long long)(AUX_PHI0 + bin) * C.plane + n.idx];
  pull_bb<S>(PopView<S>(make_pools<S>(c, C), bin, SET_G), C, SET_G, cols_of(n.x, C.nx), n.y, g);
  float d = g[0];
  for (int i = 1; i < 9; ++i) d += g[i];
  scr[(long long)n.y * C.nx + n.x] = hi + d;
}

// Compact [ny][nx] output plane of each field (phi, u_x, u_y, p, psi, rho_e),
// -1 for a field not written
struct FieldPlanes {
  int at[6];
};

// u, p, psi, rho_e of level n into the compact planes fp selects of out (and
// phi, copied from phi_pl, if selected); phi_pl: compact plane of the level-n
// order parameter written by k_fields_phi
template <class S>
__global__ void k_fields_rest(Ctx c, int inst, const float* phi_pl, float* out, FieldPlanes fp) {
  const InstConst C = c.ic[inst];
  const int bin = c.dyn[inst].bin;
  NodeIdx n;
  if (!node_of(C, n)) return;
  const long long N = (long long)C.nx * C.ny, cidx = (long long)n.y * C.nx + n.x;
  float gphx, gphy, lphi;
  stencil_at(C, phi_pl, n.x, n.y, 0, false, gphx, gphy, lphi);  // the phi plane is compact
  const float phi = phi_pl[cidx];
  const float* aux = c.fpool + C.off_f;
  const long long aidx = n.idx;
  const InstConst& Cp = C;
  float l[9], f[9];
  const Pools P = make_pools<S>(c, Cp);
  const Cols k = cols_of(n.x, C.nx);
  pull_bb<S>(PopView<S>(P, bin, SET_L), Cp, SET_L, k, n.y, l);
  pull_bb<S>(PopView<S>(P, bin, SET_F), Cp, SET_F, k, n.y, f);
  // stored l_i are relative to w_i times the charge of their source node
  const float* q_pl = aux + (long long)(AUX_Q0 + bin) * Cp.plane;
  for (int i = 0; i < 9 && S::kChargeRef; ++i) {
    const int ys = n.y - CY[i];
    const bool wall = Cp.walls && (ys < 0 || ys >= Cp.ny);
    const int xs = wall ? n.x : wrapi(n.x - CX[i], Cp.nx), yw = wall ? n.y : wrapi(ys, Cp.ny);
    l[i] += W9[i] * q_pl[(long long)yw * Cp.ldx + col_slot(xs)];
  }
  float q = 0.f, sumf = 0.f, mx = 0.f, my = 0.f;
  for (int i = 0; i < 9; ++i) {
    q += l[i];
    mx += CX[i] * f[i];
    my += CY[i] * f[i];
    if (i) sumf += f[i];
  }
  if (Cp.q_impl) {  // Eq. (66) with R of the same level, solved for q
    float gpsx, gpsy, lpsi;
    stencil_at(Cp, aux + (long long)AUX_PSI * Cp.plane, n.x, n.y, 1, true, gpsx, gpsy, lpsi);
    const float Ex = -gpsx, Ey = -gpsy - Cp.glin;  // psi plane holds psi - psi_lin
    const float eps = Cp.eps_v + phi * phi * (2.f * phi - 3.f) * Cp.deps, sig = Cp.sig_v + phi * Cp.dsig;
    const float deps = 6.f * phi * (phi - 1.f) * Cp.deps, gE = gphx * Ex + gphy * Ey;
    const float hk = 0.5f * sig / eps;
    q = (q + 0.5f * ((sig / eps) * deps * gE - Cp.dsig * gE)) / (1.f + hk);
  } else {
    q += 0.5f * aux[(long long)AUX_R * Cp.plane + aidx];
  }
  const float rho = Cp.rho_v + phi * Cp.drho;
  float ux = 0.f, uy = 0.f;
  if (Cp.enable & EN_HYDRO) {
    ux = (mx + 0.5f * aux[(long long)AUX_FX * Cp.plane + aidx]) / rho;
    uy = (my + 0.5f * aux[(long long)AUX_FY * Cp.plane + aidx]) / rho;
  }
  const float ugr = Cp.drho * (ux * gphx + uy * gphy);
  const float s0 = -W9[0] * (ux * ux + uy * uy) * (0.5f * INV_CS2);
  const float p = CS2 * INV_1MW0 * (sumf + 0.5f * ugr + rho * s0);
  const float v[6] = {phi, ux, uy, p,
                      aux[(long long)AUX_PSI * Cp.plane + aidx] + Cp.psi_b + Cp.glin * ((float)n.y + 0.5f), q};
#pragma unroll
  for (int f = 0; f < 6; ++f)
    if (fp.at[f] >= 0) out[(long long)fp.at[f] * N + cidx] = v[f];
}

}  // namespace

// ===========================================================================
// host side
// ===========================================================================
struct lbm_ehd {
  int n_inst = 0, prec = 0;
  bool conv = false;         // conventional potential scheme (every instance)
  bool any_res = false;      // some instance stops its inner loop on the Poisson residual
  hipStream_t stream = nullptr;
  std::vector<lbm_ehd_params> params;
  std::vector<InstConst> ic;
  std::vector<int4> tiles;
  lbm_ehd_launch launch{64, 64, 1, 0, 0, 0, 0, 0};
  std::vector<int> inst_band;  // per-instance band height (0: the launch shape's)
  int n_solo = 0;            // instances advanced by k_solo under the current launch shape
  hipStream_t solo_stream = nullptr;  // k_solo's stream (default priority)
  hipEvent_t ev_go = nullptr, ev_solo = nullptr;  // start of a call -> k_solo -> end of the call
  Ctx ctx{};
  int tile_cap = 0;
  float* stage = nullptr;    // workspace: 6 compact planes of the largest instance
  long long stage_elems = 0;
  float* noalloc_phi = nullptr;  // this device's copy of the fixed order-parameter array
  int bin = 0;               // buffer holding the latest post-collision g, l, f
  int status = 0;
  int* h_cnt = nullptr;      // pinned host word: instances done with the running call
  hipStream_t cap_stream = nullptr;  // stream used only to capture round graphs
  std::vector<std::pair<int, hipGraphExec_t>> graphs;  // captured round graphs by length
  bool timing = false;       // eager launches with events around each kernel
  std::vector<hipEvent_t> ev;  // 3 per round of the current chunk
  lbm_ehd_timing_t tacc{};
  ~lbm_ehd() {
    for (auto e : ev) (void)hipEventDestroy(e);
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (solo_stream) (void)hipStreamDestroy(solo_stream);
    if (ev_go) (void)hipEventDestroy(ev_go);
    if (ev_solo) (void)hipEventDestroy(ev_solo);
    if (h_cnt) (void)hipHostFree(h_cnt);
  }
};

// ---------------------------------------------------------------------------
// Fixed device array of lbm_ehd_fields_noalloc: the level-n order parameter
// of one instance, which the stencils of the other fields read.  In host code
// the name `scratch` only stands in for the symbol; its device address, one
// per device, comes from hipGetSymbolAddress at lbm_ehd_init and is kept in
// noalloc_ptr (and in the handle).
// ---------------------------------------------------------------------------
static __device__ __align__(256) float scratch[LBM_EHD_NOALLOC_MAX_NODES];

namespace {

#define HIP_OK(expr)                                    \
  do {                                                  \
    if ((expr) != hipSuccess) return LBM_EHD_E_HIP;     \
  } while (0)

int validate(const lbm_ehd_params& p) {
  if (p.nx < 1 || p.ny < 1) return LBM_EHD_E_INVAL;
  if (p.walls_y && p.ny < 3) return LBM_EHD_E_INVAL;
  if (!(p.rho_l > 0 && p.rho_v > 0 && p.mu_l > 0 && p.mu_v > 0)) return LBM_EHD_E_INVAL;
  if (!(p.eps_l > 0 && p.eps_v > 0 && p.mobility > 0 && p.width > 0 && p.gamma > 0)) return LBM_EHD_E_INVAL;
  if (!(p.sigma_l >= 0 && p.sigma_v >= 0)) return LBM_EHD_E_INVAL;
  if ((p.enable & EN_NP) && !(p.alpha_q > 0)) return LBM_EHD_E_INVAL;
  if (p.pot_max_iter < 1 || p.presolve_iters < 0 || !(p.pot_tol >= 0)) return LBM_EHD_E_INVAL;
  if (p.enable & ~15) return LBM_EHD_E_INVAL;
  if (p.pot_scheme != LBM_EHD_POT_IMPROVED && p.pot_scheme != LBM_EHD_POT_CONVENTIONAL) return LBM_EHD_E_INVAL;
  if (p.pot_scheme == LBM_EHD_POT_CONVENTIONAL && !(p.pot_chi > 0 && p.pot_chi < 1e30)) return LBM_EHD_E_INVAL;
  if (p.charge_closure != LBM_EHD_Q_LAGGED && p.charge_closure != LBM_EHD_Q_IMPLICIT) return LBM_EHD_E_INVAL;
  if (p.pot_stop != LBM_EHD_STOP_CHANGE && p.pot_stop != LBM_EHD_STOP_RESIDUAL) return LBM_EHD_E_INVAL;
  // without the Nernst-Planck set the charge is frozen, which needs a zero source
  if (!(p.enable & EN_NP) && (p.sigma_l != 0.0 || p.sigma_v != 0.0)) return LBM_EHD_E_INVAL;
  // 32-bit buffer offsets: a pool (64 plane segments per row and strip, 4 bytes) stays below 4 GiB
  if ((long long)((p.nx + STRIP - 1) / STRIP) * BLOCK_PLANES * SEG * p.ny >= (1LL << 30)) return LBM_EHD_E_INVAL;
  return LBM_EHD_OK;
}

// strips of 64 columns, the last one padded to 64 slots (see the device header)
int row_pitch(int nx) { return (nx + STRIP - 1) / STRIP * BLOCK_PLANES * SEG; }
// elements of one pool of an instance (every plane of every row)
long long pool_elems(const lbm_ehd_params& p) { return (long long)row_pitch(p.nx) * p.ny; }

// band height of an instance under a launch shape
int band_of(const lbm_ehd_launch& L, int ny) {
  return (L.small_ny > 0 && L.band_y_small > 0 && ny < L.small_ny) ? L.band_y_small : L.band_y;
}

// instances a launch shape advances by a workgroup of their own (k_solo):
// lattices of at most solo_max_nodes nodes that stop their inner loop on the
// successive change (the residual stop test needs the residual pass of the
// round path)
bool is_solo(const lbm_ehd_launch& L, const lbm_ehd_params& p) {
  return L.solo_max_nodes > 0 && (long long)p.nx * p.ny <= (long long)L.solo_max_nodes &&
         p.pot_stop == LBM_EHD_STOP_CHANGE;
}

// tiles of every instance for a launch shape and the per-instance band
// heights that replace it (ovr may be NULL; 0 entries follow the shape): the
// instances of the round path first, in instance order, then the solo ones;
// begin[i], end[i]: tile range of instance i (either may be NULL); *n_first:
// count of the first part (may be NULL); returns the count
int build_tiles(const std::vector<lbm_ehd_params>& ps, const lbm_ehd_launch& L, const std::vector<int>* ovr,
                std::vector<int4>* out, std::vector<int>* begin, std::vector<int>* end, int* n_first) {
  const int T = STRIP;  // one strip per wave
  int n = 0;
  if (begin) begin->assign(ps.size(), 0);
  if (end) end->assign(ps.size(), 0);
  if (n_first) *n_first = 0;
  for (int part = 0; part < 2; ++part) {
    if (part == 1 && n_first) *n_first = n;
    for (size_t i = 0; i < ps.size(); ++i) {
      if (is_solo(L, ps[i]) != (part == 1)) continue;
      if (begin) (*begin)[i] = n;
      const int band_y = (ovr && (*ovr)[i] > 0) ? (*ovr)[i] : band_of(L, ps[i].ny);
      for (int y0 = 0; y0 < ps[i].ny; y0 += band_y)
        for (int x0 = 0; x0 < ps[i].nx; x0 += T) {
          if (out) out->push_back(make_int4((int)i, x0, y0, std::min(y0 + band_y, ps[i].ny)));
          ++n;
        }
      if (end) (*end)[i] = n;
    }
  }
  return n;
}

struct Layout {
  size_t off_ic, off_dyn, off_tiles, off_pm, off_pp, off_pr, off_khist, off_replay, off_ctr, off_solo, off_scr,
      off_f, off_m, total;
  long long n_f, n_m, scr_elems;
  int tile_cap;
};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

Layout plan(const std::vector<lbm_ehd_params>& ps, int prec) {
  Layout L{};
  const int n = (int)ps.size();
  L.tile_cap = build_tiles(ps, lbm_ehd_launch{64, 4, 1, 0, 0, 0, 0, 0}, nullptr, nullptr, nullptr, nullptr, nullptr);
  long long nf = 0, nm = 0, scr = 0;
  for (const auto& p : ps) {
    nf += pool_elems(p);
    nm += pool_elems(p);
    scr = std::max(scr, 6LL * p.nx * p.ny);
  }
  L.n_f = nf;
  L.n_m = nm;
  L.scr_elems = std::max(scr, 2LL * 1);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = align256(o + bytes);
    return r;
  };
  L.off_ic = take(sizeof(InstConst) * n);
  L.off_dyn = take(sizeof(InstDyn) * n);
  L.off_tiles = take(sizeof(int4) * L.tile_cap);
  L.off_pm = take(sizeof(double2) * 2 * L.tile_cap);
  L.off_pp = take(sizeof(double2) * 2 * L.tile_cap);
  L.off_pr = take(sizeof(double2) * L.tile_cap);
  L.off_khist = take(sizeof(int) * (size_t)n * HIST);
  L.off_replay = take(sizeof(int) * (size_t)n * HIST);
  L.off_ctr = take(sizeof(int) * 4);
  L.off_solo = take(sizeof(int) * (size_t)n);
  L.off_scr = take(sizeof(float) * L.scr_elems);
  L.off_f = take(sizeof(float) * nf);
  L.off_m = take((prec == LBM_EHD_PREC_FP16S ? 2 : 4) * nm);
  L.total = o;
  return L;
}

float pow2_scale(double mag) {
  // power-of-two scale mapping the expected magnitude to about 64
  if (!(mag > 0)) mag = 1.0;
  const int e = (int)std::floor(std::log2(64.0 / mag));
  return std::ldexp(1.0f, std::max(-60, std::min(60, e)));
}

InstConst make_const(const lbm_ehd_params& p, long long off_f, long long off_m, const double* q0) {
  InstConst C{};
  C.off_f = off_f;
  C.off_m = off_m;
  C.nx = p.nx;
  C.ny = p.ny;
  C.ldx = row_pitch(p.nx);
  C.plane = SEG;
  C.walls = p.walls_y ? 1 : 0;
  C.enable = p.enable;
  const double cs2 = 1.0 / 3.0;
  const double beta = 12.0 * p.gamma / p.width, kappa = 3.0 * p.gamma * p.width / 2.0;
  C.rho_v = (float)p.rho_v;
  C.drho = (float)(p.rho_l - p.rho_v);
  C.mu_v = (float)p.mu_v;
  C.dmu = (float)(p.mu_l - p.mu_v);
  C.sig_v = (float)p.sigma_v;
  C.dsig = (float)(p.sigma_l - p.sigma_v);
  C.eps_v = (float)p.eps_v;
  C.deps = (float)(p.eps_v - p.eps_l);
  C.beta4 = (float)(4.0 * beta);
  C.kappa = (float)kappa;
  const double tau_g = 0.5 + p.mobility / cs2, tau_h = 0.5 + p.eps_v / cs2;
  const double tau_l = 0.5 + ((p.enable & EN_NP) ? p.alpha_q : 1.0) / cs2;
  C.inv_tau_g = (float)(1.0 / tau_g);
  C.inv_tau_h = (float)(1.0 / tau_h);
  C.inv_tau_l = (float)(1.0 / tau_l);
  C.fac_l = (float)(1.0 - 0.5 / tau_l);
  C.cs2_tau_h = (float)(cs2 * tau_h);
  if (p.pot_scheme == LBM_EHD_POT_CONVENTIONAL) {
    C.conv_k = (float)(1.0 / (p.pot_chi * cs2));
    C.conv_src = (float)(0.125 / p.pot_chi);
  }
  const double wet = std::sqrt(2.0 * beta / kappa);
  const double d2r = M_PI / 180.0;
  C.wet_b = (float)(wet * (std::cos(p.theta_bottom_deg * d2r) + p.cos_shift_bottom));
  C.wet_t = (float)(wet * (std::cos(p.theta_top_deg * d2r) + p.cos_shift_top));
  C.psi_b = (float)(p.walls_y ? p.psi_bottom : 0.0);
  C.psi_t = (float)(p.walls_y ? p.psi_top : 0.0);
  C.glin = (float)(p.walls_y ? (p.psi_top - p.psi_bottom) / p.ny : 0.0);
  C.q_impl = p.charge_closure == LBM_EHD_Q_IMPLICIT ? 1 : 0;
  C.tol = p.pot_tol;
  C.max_iter = p.pot_max_iter;
  C.presolve_iters = p.presolve_iters;
  C.pot_stop = p.pot_stop == LBM_EHD_STOP_RESIDUAL ? 1 : 0;
  // FP16 moving populations: (pop - offset) / w_i times a power-of-two scale
  // chosen from the expected magnitude of that quotient for each set
  const double dpsi = p.walls_y ? std::fabs(p.psi_top - p.psi_bottom) : 0.0;
  const double E0 = std::max(dpsi / p.ny, 1e-6);
  const double eps_ratio = std::max(p.eps_l / p.eps_v, p.eps_v / p.eps_l);
  double qmax = 0.0;
  for (long long k = 0; k < (long long)p.nx * p.ny; ++k) qmax = std::max(qmax, std::fabs(q0[k]));
  const double q_est = std::max(qmax, std::max(p.eps_l, p.eps_v) * E0 / p.width);
  const double mu_est = std::max(0.2 * beta, std::fabs(p.eps_l - p.eps_v) * E0 * E0);
  const double mu_min = std::min(p.mu_l, p.mu_v), rho_max = std::max(p.rho_l, p.rho_v);
  const double u_est = std::max(std::max(p.eps_l, p.eps_v) * E0 * E0 * p.ny / (8.0 * mu_min), 1e-6);
  const double p_est = std::max(p.gamma * 8.0 / std::min(p.nx, p.ny), p.eps_v * E0 * E0);
  const double mag[4] = {mu_est, q_est, 3.0 * rho_max * u_est + 3.0 * p_est, E0 * eps_ratio};
  for (int k = 0; k < 4; ++k) {
    C.scale[k] = pow2_scale(mag[k]);
    C.inv_scale[k] = 1.0f / C.scale[k];
    const float w[2] = {1.f / 9.f, 1.f / 36.f}, iw[2] = {9.f, 36.f};
    for (int j = 0; j < 2; ++j) {
      C.dec[k][j] = w[j] * C.inv_scale[k];
      C.enc[k][j] = iw[j] * C.scale[k];
    }
  }
  return C;
}

int refresh_status(lbm_ehd* s) {
  // sticky per-instance bits -> handle status
  std::vector<InstDyn> d(s->n_inst);
  HIP_OK(hipStreamSynchronize(s->stream));
  HIP_OK(hipMemcpy(d.data(), s->ctx.dyn, sizeof(InstDyn) * s->n_inst, hipMemcpyDeviceToHost));
  int diverged = 0, capped = 0;
  for (const auto& x : d) {
    diverged += (x.status & 2) ? 1 : 0;
    capped += (x.status & 1) ? 1 : 0;
  }
  const int st = diverged == s->n_inst ? LBM_EHD_E_DIVERGED
                 : diverged          ? LBM_EHD_W_DIVERGED
                 : capped            ? LBM_EHD_W_NOT_CONVERGED
                                     : LBM_EHD_OK;
  // fatal codes stay; among warnings the larger one wins
  if (s->status >= 0 && (st < 0 || st > s->status)) s->status = st;
  return s->status;
}

// enqueues R rounds (round + finalize) on stream st; in timing mode with an
// event before, between and after the two kernels of every round
template <class S>
int enqueue_rounds(lbm_ehd* s, hipStream_t st, int R) {
  const int nt = std::max(s->ctx.n_ns_tiles, 1);
  const bool tm = s->timing && st == s->stream;
  if (tm)
    while ((int)s->ev.size() < 3 * R) {
      hipEvent_t e;
      HIP_OK(hipEventCreate(&e));
      s->ev.push_back(e);
    }
  for (int r = 0; r < R; ++r) {
    if (tm) HIP_OK(hipEventRecord(s->ev[3 * r], st));
    const int wpb = s->launch.block_x / WAVE;
    hipLaunchKernelGGL(k_round<S>, dim3((nt + wpb - 1) / wpb), dim3(s->launch.block_x), 0, st, s->ctx);
    if (tm) HIP_OK(hipEventRecord(s->ev[3 * r + 1], st));
    if (s->any_res) hipLaunchKernelGGL(k_residual, dim3(s->ctx.n_tiles), dim3(WAVE), 0, st, s->ctx, -1);
    hipLaunchKernelGGL(k_finalize, dim3(s->n_inst), dim3(FIN_THREADS), 0, st, s->ctx);
    if (tm) HIP_OK(hipEventRecord(s->ev[3 * r + 2], st));
  }
  return LBM_EHD_OK;
}

// adds the event times of the last timed round (stream synchronised); n_main /
// n_pot: instances that ran a main pass / an inner iteration in it
int collect_times(lbm_ehd* s, int n_main, int n_pot) {
  float a = 0.f, b = 0.f;
  HIP_OK(hipEventElapsedTime(&a, s->ev[0], s->ev[1]));
  HIP_OK(hipEventElapsedTime(&b, s->ev[1], s->ev[2]));
  lbm_ehd_timing_t& T = s->tacc;
  T.round_ms += a;
  T.finalize_ms += b;
  T.round_launches += 1;
  T.finalize_launches += 1;
  if (n_pot == 0) {
    T.main_round_ms += a;
    T.main_rounds += 1;
  } else if (n_main == 0) {
    T.pot_round_ms += a;
    T.pot_rounds += 1;
  }
  T.main_passes += n_main;
  T.inner_iterations += n_pot;
  return LBM_EHD_OK;
}

// graph of R rounds, captured once per R on the library's own capture stream
template <class S>
int round_graph(lbm_ehd* s, int R, hipGraphExec_t* out) {
  for (auto& g : s->graphs)
    if (g.first == R) {
      *out = g.second;
      return LBM_EHD_OK;
    }
  if (!s->cap_stream) HIP_OK(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  HIP_OK(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
  (void)enqueue_rounds<S>(s, s->cap_stream, R);
  HIP_OK(hipStreamEndCapture(s->cap_stream, &graph));
  hipGraphExec_t exec = nullptr;
  const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return LBM_EHD_E_HIP;
  s->graphs.emplace_back(R, exec);
  *out = exec;
  return LBM_EHD_OK;
}

// Runs rounds until every instance has finished n_target outer steps (or the
// initial potential solve).  Host-steered: one round per check.  Device loop:
// graph-captured chunks of rounds, one check per chunk; rounds beyond an
// instance's target are no-ops for it.
template <class S>
int run_rounds(lbm_ehd* s, int n_target, bool presolve) {
  hipLaunchKernelGGL(k_begin, dim3(1), dim3(256), 0, s->stream, s->ctx, n_target, presolve ? 1 : 0);
  HIP_OK(hipGetLastError());
  if (s->n_solo > 0) {
    // the solo instances' whole call, on a stream of its own beside the rounds
    if (!s->solo_stream) HIP_OK(hipStreamCreateWithFlags(&s->solo_stream, hipStreamNonBlocking));
    if (!s->ev_go) HIP_OK(hipEventCreateWithFlags(&s->ev_go, hipEventDisableTiming));
    if (!s->ev_solo) HIP_OK(hipEventCreateWithFlags(&s->ev_solo, hipEventDisableTiming));
    HIP_OK(hipEventRecord(s->ev_go, s->stream));
    HIP_OK(hipStreamWaitEvent(s->solo_stream, s->ev_go, 0));
    hipLaunchKernelGGL(k_solo<S>, dim3(s->n_solo), dim3(FIN_THREADS), 0, s->solo_stream, s->ctx);
    HIP_OK(hipGetLastError());
    HIP_OK(hipEventRecord(s->ev_solo, s->solo_stream));
  }
  const int n_round = s->n_inst - s->n_solo;  // instances of the round path
  const bool dev = s->launch.device_loop && !presolve;
  int chunk = 0, pending = 0, seen_main = 0, seen_pot = 0;
  for (;;) {
    HIP_OK(hipMemcpyAsync(s->h_cnt, s->ctx.counters, 3 * sizeof(int), hipMemcpyDeviceToHost, s->stream));
    HIP_OK(hipStreamSynchronize(s->stream));
    if (pending) {
      const int rc = collect_times(s, s->h_cnt[1] - seen_main, s->h_cnt[2] - seen_pot);
      if (rc != LBM_EHD_OK) return rc;
      pending = 0;
    }
    seen_main = s->h_cnt[1];
    seen_pot = s->h_cnt[2];
    if (*s->h_cnt >= n_round) break;
    // device loop: the first chunk is sized for n_target steps of one inner
    // iteration each, later chunks for the remaining longer loops; timing
    // mode steps one round per check so that no idle round is timed
    const int auto_first = std::min(2 * n_target + 2, 1024);
    const int auto_next = std::max(8, std::min(auto_first / 8, 256));
    const int rpg = s->launch.rounds_per_graph;
    const int R = (!dev || s->timing) ? 1 : chunk == 0 ? (rpg > 0 ? rpg : auto_first) : (rpg > 0 ? rpg : auto_next);
    if (dev && !s->timing) {
      hipGraphExec_t g = nullptr;
      const int rc = round_graph<S>(s, R, &g);
      if (rc != LBM_EHD_OK) return rc;
      HIP_OK(hipGraphLaunch(g, s->stream));
    } else {
      const int rc = enqueue_rounds<S>(s, s->stream, R);
      if (rc != LBM_EHD_OK) return rc;
      HIP_OK(hipGetLastError());
      if (s->timing) pending = 1;  // R == 1 in timing mode
    }
    ++chunk;
  }
  // later work on the handle's stream (and its synchronisation) follows the solo instances
  if (s->n_solo > 0) HIP_OK(hipStreamWaitEvent(s->stream, s->ev_solo, 0));
  return LBM_EHD_OK;
}

template <class S>
int do_steps(lbm_ehd* s, int n_steps) {
  return run_rounds<S>(s, n_steps, false);
}

// calls f with the storage trait of the handle (precision x potential scheme)
template <class F>
int with_store(const lbm_ehd* s, F&& f) {
  if (s->prec == LBM_EHD_PREC_FP16S) return s->conv ? f(ConvPot<StoreF16S>{}) : f(StoreF16S{});
  return s->conv ? f(ConvPot<StoreF32>{}) : f(StoreF32{});
}

void drop_graphs(lbm_ehd* s) {
  for (auto& g : s->graphs) (void)hipGraphExecDestroy(g.second);
  s->graphs.clear();
}

int apply_launch(lbm_ehd* s, const lbm_ehd_launch& L) {
  if (L.block_x != WAVE && L.block_x != 2 * WAVE && L.block_x != 4 * WAVE) return LBM_EHD_E_INVAL;
  if (L.band_y < 4 || L.band_y > 1024 || L.rounds_per_graph < 0 || L.rounds_per_graph > 100000 ||
      (L.device_loop != 0 && L.device_loop != 1) || L.small_ny < 0 ||
      (L.band_y_small != 0 && (L.band_y_small < 4 || L.band_y_small > 1024)) || L.solo_max_nodes < 0 ||
      (L.stagger != 0 && L.stagger != 1))
    return LBM_EHD_E_INVAL;
  std::vector<int4> tiles;
  std::vector<int> begin, end, solo;
  int n_first = 0;
  const int n = build_tiles(s->params, L, &s->inst_band, &tiles, &begin, &end, &n_first);
  if (n > s->tile_cap) return LBM_EHD_E_INVAL;
  // host-side bounds check of every tile against its instance, and of the
  // two parts of the list (the round path's instances, then the solo ones)
  for (int t = 0; t < n; ++t) {
    const int4 q = tiles[t];
    const auto& p = s->params[q.x];
    if (q.y < 0 || q.y >= p.nx || q.z < 0 || q.w > p.ny || q.z >= q.w) return LBM_EHD_E_INVAL;
    if (is_solo(L, p) != (t >= n_first)) return LBM_EHD_E_INVAL;
  }
  // staggered start: in instance order, each round-path instance joins the
  // group with fewer nodes so far (the groups alternate along the work list)
  long long grp[2] = {0, 0};
  for (int i = 0; i < s->n_inst; ++i) {
    s->ic[i].tile_begin = begin[i];
    s->ic[i].tile_end = end[i];
    s->ic[i].owner_tile = begin[i];
    s->ic[i].solo = is_solo(L, s->params[i]) ? 1 : 0;
    s->ic[i].stagger = 0;
    if (s->ic[i].solo) {
      solo.push_back(i);
    } else if (L.stagger) {
      const int g = grp[1] < grp[0] ? 1 : 0;
      grp[g] += (long long)s->params[i].nx * s->params[i].ny;
      s->ic[i].stagger = g;
    }
  }
  HIP_OK(hipMemcpyAsync(const_cast<int4*>(s->ctx.tiles), tiles.data(), sizeof(int4) * n, hipMemcpyHostToDevice, s->stream));
  HIP_OK(hipMemcpyAsync(const_cast<InstConst*>(s->ctx.ic), s->ic.data(), sizeof(InstConst) * s->n_inst,
                        hipMemcpyHostToDevice, s->stream));
  if (!solo.empty())
    HIP_OK(hipMemcpyAsync(const_cast<int*>(s->ctx.solo_list), solo.data(), sizeof(int) * solo.size(),
                          hipMemcpyHostToDevice, s->stream));
  HIP_OK(hipStreamSynchronize(s->stream));
  drop_graphs(s);
  s->tiles.swap(tiles);
  s->ctx.n_tiles = n;
  s->ctx.n_ns_tiles = n_first;
  s->ctx.n_solo = (int)solo.size();
  s->n_solo = (int)solo.size();
  s->launch = L;
  return LBM_EHD_OK;
}

// the two field kernels of instance inst on the handle's stream: level-n phi
// into the compact plane phi_pl, then the fields fp selects into out
void enqueue_fields(lbm_ehd* s, int inst, float* phi_pl, float* out, const FieldPlanes& fp) {
  const InstConst& C = s->ic[inst];
  const long long N = (long long)C.nx * C.ny;
  const int TB = 256;
  const unsigned nb = (unsigned)((N + TB - 1) / TB);
  if (s->prec == LBM_EHD_PREC_FP16S) {
    hipLaunchKernelGGL(k_fields_phi<StoreF16S>, dim3(nb), dim3(TB), 0, s->stream, s->ctx, inst, phi_pl);
    hipLaunchKernelGGL(k_fields_rest<StoreF16S>, dim3(nb), dim3(TB), 0, s->stream, s->ctx, inst,
                       (const float*)phi_pl, out, fp);
  } else {
    hipLaunchKernelGGL(k_fields_phi<StoreF32>, dim3(nb), dim3(TB), 0, s->stream, s->ctx, inst, phi_pl);
    hipLaunchKernelGGL(k_fields_rest<StoreF32>, dim3(nb), dim3(TB), 0, s->stream, s->ctx, inst,
                       (const float*)phi_pl, out, fp);
  }
}

constexpr int MAX_DEVICES = 64;
std::mutex noalloc_mu;
void* noalloc_ptr[MAX_DEVICES] = {};

// address of this device's copy of scratch (the current device), resolved
// once per device; NULL if the runtime cannot give it
float* noalloc_scratch_here() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(noalloc_mu);
  if (!noalloc_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    noalloc_ptr[dev] = p;
  }
  return (float*)noalloc_ptr[dev];
}

}  // namespace

extern "C" {

int lbm_ehd_workspace_bytes(const lbm_ehd_params* p, int32_t n_inst, int32_t prec, size_t* bytes) {
  if (!p || n_inst < 1 || !bytes || (prec != LBM_EHD_PREC_FP32 && prec != LBM_EHD_PREC_FP16S))
    return LBM_EHD_E_INVAL;
  std::vector<lbm_ehd_params> ps(p, p + n_inst);
  for (const auto& x : ps)
    if (validate(x) != LBM_EHD_OK || x.pot_scheme != ps[0].pot_scheme) return LBM_EHD_E_INVAL;
  *bytes = plan(ps, prec).total;
  return LBM_EHD_OK;
}

int lbm_ehd_init(const lbm_ehd_params* p, int32_t n_inst, int32_t prec, const double* phi0, const double* q0,
                 const double* ux0, const double* uy0, void* d_workspace, size_t workspace_bytes, void* stream,
                 lbm_ehd** out) {
  if (!out) return LBM_EHD_E_INVAL;
  *out = nullptr;
  if (!p || n_inst < 1 || !phi0 || !q0 || (prec != LBM_EHD_PREC_FP32 && prec != LBM_EHD_PREC_FP16S))
    return LBM_EHD_E_INVAL;
  if ((ux0 == nullptr) != (uy0 == nullptr)) return LBM_EHD_E_INVAL;
  std::vector<lbm_ehd_params> ps(p, p + n_inst);
  for (const auto& x : ps)
    if (validate(x) != LBM_EHD_OK || x.pot_scheme != ps[0].pot_scheme) return LBM_EHD_E_INVAL;
  const Layout L = plan(ps, prec);
  if (!d_workspace || workspace_bytes < L.total || ((uintptr_t)d_workspace & 255)) return LBM_EHD_E_WORKSPACE;

  lbm_ehd* s = new (std::nothrow) lbm_ehd();
  if (!s) return LBM_EHD_E_INVAL;
  s->n_inst = n_inst;
  s->prec = prec;
  s->conv = ps[0].pot_scheme == LBM_EHD_POT_CONVENTIONAL;
  for (const auto& x : ps) s->any_res = s->any_res || x.pot_stop == LBM_EHD_STOP_RESIDUAL;
  s->stream = (hipStream_t)stream;
  s->params = ps;
  s->inst_band.assign(n_inst, 0);
  s->tile_cap = L.tile_cap;
  char* ws = (char*)d_workspace;
  Ctx& c = s->ctx;
  c.ic = (const InstConst*)(ws + L.off_ic);
  c.dyn = (InstDyn*)(ws + L.off_dyn);
  c.tiles = (const int4*)(ws + L.off_tiles);
  c.part_main = (double2*)(ws + L.off_pm);
  c.part_pot = (double2*)(ws + L.off_pp);
  c.part_floor = (double*)(ws + L.off_pp + sizeof(double2) * L.tile_cap);
  c.part_res = (double2*)(ws + L.off_pr);
  c.khist = (int*)(ws + L.off_khist);
  c.replay = (const int*)(ws + L.off_replay);
  c.counters = (int*)(ws + L.off_ctr);
  c.solo_list = (const int*)(ws + L.off_solo);
  c.fpool = (float*)(ws + L.off_f);
  c.mpool = (void*)(ws + L.off_m);
  c.n_inst = n_inst;
  s->stage = (float*)(ws + L.off_scr);
  s->stage_elems = L.scr_elems;

  auto fail = [&](int code) {
    delete s;
    return code;
  };
  // device address of the fixed array of lbm_ehd_fields_noalloc on this
  // device (resolved at the first init on each device)
  s->noalloc_phi = noalloc_scratch_here();
  if (hipHostMalloc((void**)&s->h_cnt, 4 * sizeof(int), hipHostMallocDefault) != hipSuccess) return fail(LBM_EHD_E_HIP);
  // constants and offsets
  long long of = 0, om = 0, node0 = 0;
  s->ic.resize(n_inst);
  for (int i = 0; i < n_inst; ++i) {
    s->ic[i] = make_const(ps[i], of, om, q0 + node0);
    of += pool_elems(ps[i]);
    om += pool_elems(ps[i]);
    node0 += (long long)ps[i].nx * ps[i].ny;
  }
  // zero all bookkeeping and state
  if (hipMemsetAsync(d_workspace, 0, L.total, s->stream) != hipSuccess) return fail(LBM_EHD_E_HIP);
  int rc = apply_launch(s, s->launch);
  if (rc != LBM_EHD_OK) return fail(rc);

  // upload phi0 (both phi planes), q0 per instance into the aux planes
  node0 = 0;
  std::vector<float> tmp;
  for (int i = 0; i < n_inst; ++i) {
    const InstConst& C = s->ic[i];
    const long long N = (long long)C.nx * C.ny;
    tmp.resize(N);
    const int TB = 256;
    const unsigned nb = (unsigned)((N + TB - 1) / TB);
    const double* srcs[4] = {phi0 + node0, phi0 + node0, q0 + node0, q0 + node0};
    const int planes[4] = {AUX_PHI0, AUX_PHI1, AUX_Q0, AUX_Q1};
    for (int k = 0; k < 4; ++k) {
      for (long long j = 0; j < N; ++j) tmp[j] = (float)srcs[k][j];
      if (hipMemcpy(s->stage, tmp.data(), sizeof(float) * N, hipMemcpyHostToDevice) != hipSuccess)
        return fail(LBM_EHD_E_HIP);
      hipLaunchKernelGGL(k_put_plane, dim3(nb), dim3(TB), 0, s->stream, c.fpool + C.off_f + planes[k] * C.plane,
                         s->stage, C.nx, C.ny, C.ldx);
      if (hipStreamSynchronize(s->stream) != hipSuccess) return fail(LBM_EHD_E_HIP);
    }
    node0 += N;
  }
  auto init_all = [&](auto tag) -> int {
    using S = decltype(tag);
    const int TB = 256;
    for (int i = 0; i < n_inst; ++i) {
      const InstConst& C = s->ic[i];
      const unsigned nb = (unsigned)(((long long)C.nx * C.ny + TB - 1) / TB);
      hipLaunchKernelGGL(k_init_h<S>, dim3(nb), dim3(TB), 0, s->stream, c, i);
    }
    if (hipGetLastError() != hipSuccess) return LBM_EHD_E_HIP;
    const int r = run_rounds<S>(s, 0, true);  // initial potential solve
    if (r != LBM_EHD_OK) return r;
    long long n0 = 0;
    for (int i = 0; i < n_inst; ++i) {
      const InstConst& C = s->ic[i];
      const long long N = (long long)C.nx * C.ny;
      std::vector<float> u(3 * N, 0.f);
      for (long long j = 0; j < N; ++j) {
        if (ux0) {
          u[j] = (float)ux0[n0 + j];
          u[N + j] = (float)uy0[n0 + j];
        }
        u[2 * N + j] = (float)(phi0[n0 + j] - (double)(float)phi0[n0 + j]);
      }
      if (hipMemcpy(s->stage, u.data(), sizeof(float) * 3 * N, hipMemcpyHostToDevice) != hipSuccess)
        return LBM_EHD_E_HIP;
      const unsigned nb = (unsigned)((N + TB - 1) / TB);
      hipLaunchKernelGGL(k_init_pops<S>, dim3(nb), dim3(TB), 0, s->stream, c, i, (const float*)s->stage,
                         ux0 ? 1 : 0);
      if (hipStreamSynchronize(s->stream) != hipSuccess) return LBM_EHD_E_HIP;
      n0 += N;
    }
    return LBM_EHD_OK;
  };
  rc = with_store(s, init_all);
  if (rc != LBM_EHD_OK) return fail(rc);
  // every instance diverged in the initial solve: no handle is returned
  rc = refresh_status(s);
  if (rc < 0) return fail(rc);
  *out = s;
  return LBM_EHD_OK;
}

int lbm_ehd_step(lbm_ehd* s, int32_t n_steps) {
  if (!s || n_steps < 0) return LBM_EHD_E_INVAL;
  if (s->status < 0) return s->status;
  if (n_steps == 0) return s->status;
  const int rc = with_store(s, [&](auto tag) { return do_steps<decltype(tag)>(s, n_steps); });
  if (rc != LBM_EHD_OK) {
    s->status = rc;
    return rc;
  }
  return refresh_status(s);
}

int lbm_ehd_sync(lbm_ehd* s) {
  if (!s) return LBM_EHD_E_INVAL;
  return refresh_status(s);
}

int lbm_ehd_fields(lbm_ehd* s, int32_t inst, uint32_t mask, float* out, int32_t out_on_device) {
  if (!s || inst < 0 || inst >= s->n_inst || !out || (mask & ~63u) || mask == 0) return LBM_EHD_E_INVAL;
  const int st = refresh_status(s);
  if (st == LBM_EHD_E_HIP) return st;
  const InstConst& C = s->ic[inst];
  const long long N = (long long)C.nx * C.ny;
  // every field into its plane of the staging area (phi is already in plane 0)
  const FieldPlanes fp{{-1, 1, 2, 3, 4, 5}};
  enqueue_fields(s, inst, s->stage, s->stage, fp);
  HIP_OK(hipGetLastError());
  int k = 0;
  for (int f = 0; f < 6; ++f) {
    if (!(mask & (1u << f))) continue;
    HIP_OK(hipMemcpyAsync(out + (long long)k * N, s->stage + (long long)f * N, sizeof(float) * N,
                          out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s->stream));
    ++k;
  }
  HIP_OK(hipStreamSynchronize(s->stream));
  return LBM_EHD_OK;
}

int lbm_ehd_fields_noalloc(lbm_ehd* s, int32_t inst, uint32_t mask, float* d_out) {
  if (!s || inst < 0 || inst >= s->n_inst || !d_out || (mask & ~63u) || mask == 0) return LBM_EHD_E_INVAL;
  if (s->status < 0) return s->status;
  const InstConst& C = s->ic[inst];
  if ((long long)C.nx * C.ny > LBM_EHD_NOALLOC_MAX_NODES) return LBM_EHD_E_INVAL;
  if (!s->noalloc_phi) return LBM_EHD_E_STATE;
  FieldPlanes fp{{-1, -1, -1, -1, -1, -1}};
  int k = 0;
  for (int f = 0; f < 6; ++f)
    if (mask & (1u << f)) fp.at[f] = k++;
  enqueue_fields(s, inst, s->noalloc_phi, d_out, fp);
  HIP_OK(hipGetLastError());
  return LBM_EHD_OK;
}

int lbm_ehd_residual(lbm_ehd* s, int32_t inst, double* out) {
  if (!s || inst < 0 || inst >= s->n_inst || !out) return LBM_EHD_E_INVAL;
  if (s->status < 0) return s->status;
  HIP_OK(hipStreamSynchronize(s->stream));
  const InstConst& C = s->ic[inst];
  hipLaunchKernelGGL(k_residual, dim3(s->ctx.n_tiles), dim3(WAVE), 0, s->stream, s->ctx, inst);
  HIP_OK(hipGetLastError());
  const int n = C.tile_end - C.tile_begin;
  std::vector<double2> part(n);
  HIP_OK(hipMemcpyAsync(part.data(), s->ctx.part_res + C.tile_begin, sizeof(double2) * n, hipMemcpyDeviceToHost,
                        s->stream));
  HIP_OK(hipStreamSynchronize(s->stream));
  double a = 0.0, b = 0.0;
  for (const auto& v : part) {
    a += v.x;
    b += v.y;
  }
  const double floor_den = 1e-300 * (double)C.nx * (double)C.ny;
  *out = std::sqrt(a / (b > floor_den ? b : floor_den));
  return LBM_EHD_OK;
}

int lbm_ehd_stats(lbm_ehd* s, int32_t inst, lbm_ehd_stats_t* out) {
  if (!s || inst < 0 || inst >= s->n_inst || !out) return LBM_EHD_E_INVAL;
  refresh_status(s);
  InstDyn d;
  HIP_OK(hipMemcpy(&d, s->ctx.dyn + inst, sizeof(InstDyn), hipMemcpyDeviceToHost));
  out->steps = d.steps;
  out->total_iters = d.total_iters;
  out->presolve_iters = d.presolve_k;
  out->last_iters = d.k;
  out->last_rel_change = d.last_r;
  out->sum_phi = d.sum_phi;
  out->sum_q = d.sum_q;
  out->status = (d.status & 2) ? LBM_EHD_E_DIVERGED : (d.status & 1) ? LBM_EHD_W_NOT_CONVERGED : LBM_EHD_OK;
  out->floor_stops = d.floor_stops;
  out->residual = s->ic[inst].pot_stop ? d.last_res : NAN;
  return LBM_EHD_OK;
}

int lbm_ehd_k_history(lbm_ehd* s, int32_t inst, int32_t* out, int32_t max) {
  if (!s || inst < 0 || inst >= s->n_inst || !out || max < 0) return LBM_EHD_E_INVAL;
  refresh_status(s);
  InstDyn d;
  HIP_OK(hipMemcpy(&d, s->ctx.dyn + inst, sizeof(InstDyn), hipMemcpyDeviceToHost));
  std::vector<int> ring(HIST);
  HIP_OK(hipMemcpy(ring.data(), s->ctx.khist + (long long)inst * HIST, sizeof(int) * HIST, hipMemcpyDeviceToHost));
  const long long total = d.steps + 1;
  const long long first = std::max(0LL, total - HIST);
  int n = 0;
  for (long long j = first; j < total && n < max; ++j) out[n++] = ring[j % HIST];
  return n;
}

int lbm_ehd_set_replay(lbm_ehd* s, int32_t inst, const int32_t* iters, int32_t n) {
  if (!s || inst < 0 || inst >= s->n_inst || n < 0 || n > HIST || (n > 0 && !iters)) return LBM_EHD_E_INVAL;
  for (int j = 0; j < n; ++j)
    if (iters[j] < 1) return LBM_EHD_E_INVAL;
  HIP_OK(hipStreamSynchronize(s->stream));
  if (n > 0)
    HIP_OK(hipMemcpy(const_cast<int*>(s->ctx.replay) + (long long)inst * HIST, iters, sizeof(int) * n,
                     hipMemcpyHostToDevice));
  InstDyn d;
  HIP_OK(hipMemcpy(&d, s->ctx.dyn + inst, sizeof(InstDyn), hipMemcpyDeviceToHost));
  d.replay_pos = 0;
  d.replay_n = n;
  HIP_OK(hipMemcpy(s->ctx.dyn + inst, &d, sizeof(InstDyn), hipMemcpyHostToDevice));
  return LBM_EHD_OK;
}

int lbm_ehd_set_launch(lbm_ehd* s, const lbm_ehd_launch* cfg) {
  if (!s || !cfg) return LBM_EHD_E_INVAL;
  HIP_OK(hipStreamSynchronize(s->stream));
  const lbm_ehd_launch old = s->launch;
  const int rc = apply_launch(s, *cfg);
  if (rc != LBM_EHD_OK) apply_launch(s, old);
  return rc;
}

int lbm_ehd_get_launch(const lbm_ehd* s, lbm_ehd_launch* cfg) {
  if (!s || !cfg) return LBM_EHD_E_INVAL;
  *cfg = s->launch;
  return LBM_EHD_OK;
}

int lbm_ehd_set_instance_band(lbm_ehd* s, int32_t inst, int32_t band_y) {
  if (!s || inst < 0 || inst >= s->n_inst || (band_y != 0 && (band_y < 4 || band_y > 1024))) return LBM_EHD_E_INVAL;
  HIP_OK(hipStreamSynchronize(s->stream));
  const int old = s->inst_band[inst];
  s->inst_band[inst] = band_y;
  const int rc = apply_launch(s, s->launch);
  if (rc != LBM_EHD_OK) {
    s->inst_band[inst] = old;
    apply_launch(s, s->launch);
  }
  return rc;
}

int lbm_ehd_get_instance_band(const lbm_ehd* s, int32_t inst, int32_t* band_y) {
  if (!s || inst < 0 || inst >= s->n_inst || !band_y) return LBM_EHD_E_INVAL;
  *band_y = s->inst_band[inst] > 0 ? s->inst_band[inst] : band_of(s->launch, s->params[inst].ny);
  return LBM_EHD_OK;
}

int lbm_ehd_autotune(lbm_ehd* s, int32_t trial_steps, lbm_ehd_launch* out) {
  if (!s || trial_steps < 1 || trial_steps > 10000) return LBM_EHD_E_INVAL;
  if (s->status < 0) return s->status;
  // instances below small_ny rows get their own band (their inner loops are
  // latency-bound); the larger ones the other
  constexpr int SMALL_NY = 160;
  bool has_small = false, has_large = false;
  for (const auto& p : s->params) (p.ny < SMALL_NY ? has_small : has_large) = true;
  const std::vector<int> large = has_large ? std::vector<int>{16, 32, 64} : std::vector<int>{s->launch.band_y};
  const std::vector<int> small = has_small ? std::vector<int>{4, 8, 16} : std::vector<int>{0};
  // one candidate: the first call captures its round graphs, the second is timed
  // (a stepping call returns once the rounds are done; the solo instances'
  // kernel may still run, and the handle's stream waits for it: both clock
  // readings follow a synchronisation of that stream, so the solo kernel's
  // whole time counts)
  auto timed = [&](double* t) {
    auto trial = [&](auto tag) { return do_steps<decltype(tag)>(s, trial_steps); };
    int rc = with_store(s, trial);
    if (rc != LBM_EHD_OK) return s->status = rc;
    if (hipStreamSynchronize(s->stream) != hipSuccess) return s->status = LBM_EHD_E_HIP;
    const auto t0 = std::chrono::steady_clock::now();
    rc = with_store(s, trial);
    if (rc != LBM_EHD_OK) return s->status = rc;
    if (hipStreamSynchronize(s->stream) != hipSuccess) return s->status = LBM_EHD_E_HIP;
    *t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return (int)LBM_EHD_OK;
  };
  auto read_dyn = [&](std::vector<InstDyn>* d) {
    d->resize(s->n_inst);
    if (hipMemcpyAsync(d->data(), s->ctx.dyn, sizeof(InstDyn) * s->n_inst, hipMemcpyDeviceToHost, s->stream) !=
            hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess)
      return (int)LBM_EHD_E_HIP;
    return (int)LBM_EHD_OK;
  };
  std::fill(s->inst_band.begin(), s->inst_band.end(), 0);
  // mean inner iterations per step of every instance, over trial steps on
  // the starting shape
  std::vector<InstDyn> d0, d1;
  int rc = apply_launch(s, s->launch);
  if (rc != LBM_EHD_OK) return rc;
  rc = read_dyn(&d0);
  if (rc != LBM_EHD_OK) return rc;
  double t_start = 0.;
  rc = timed(&t_start);
  if (rc != LBM_EHD_OK) return rc;
  rc = read_dyn(&d1);
  if (rc != LBM_EHD_OK) return rc;
  std::vector<double> kbar(s->n_inst, 0.);
  double kmax = 0.;
  for (int i = 0; i < s->n_inst; ++i) {
    const long long ds = d1[i].steps - d0[i].steps;
    if (ds > 0 && !(d1[i].status & 2)) kbar[i] = (double)(d1[i].total_iters - d0[i].total_iters) / (double)ds;
    kmax = std::max(kmax, kbar[i]);
  }
  // The instance with the longest inner loops sets the number of rounds of a
  // step; in most of them its tiles run on an otherwise idle device, where
  // the time of a round is the row-by-row chain of one band.  Shorter bands
  // for the slowest instances shorten those rounds at little cost in the
  // others, where they add halo rows of a few lattices only: 4 rows for the
  // instances at 0.8 of the longest mean loop or above, 8 rows for the others
  // at half of it or above (never longer than the band the shape gives).
  std::vector<int> own(s->n_inst, 0);
  for (int i = 0; i < s->n_inst && kmax >= 2.; ++i) {
    const double k = kbar[i] >= 2. ? kbar[i] / kmax : 0.;
    own[i] = k >= 0.8 ? 4 : (k >= 0.5 ? 8 : 0);
  }
  auto set_own = [&](const lbm_ehd_launch& L, bool on) {
    for (int i = 0; i < s->n_inst; ++i)
      s->inst_band[i] = on && own[i] > 0 && own[i] < band_of(L, s->params[i].ny) ? own[i] : 0;
  };
  // the shape search runs with those bands in place
  lbm_ehd_launch best = s->launch;
  double best_t = 1e300;
  for (int bl : large)
    for (int bs : small) {
      lbm_ehd_launch L = s->launch;
      L.band_y = has_large ? bl : (bs > 0 ? bs : L.band_y);
      L.band_y_small = has_small && has_large ? bs : 0;
      L.small_ny = has_small && has_large ? SMALL_NY : 0;
      set_own(L, true);
      rc = apply_launch(s, L);
      if (rc != LBM_EHD_OK) return rc;
      double t = 0.;
      rc = timed(&t);
      if (rc != LBM_EHD_OK) return rc;
      if (t < best_t) {
        best_t = t;
        best = L;
      }
    }
  // and they stay only if the chosen shape runs faster with them than without
  set_own(best, false);
  rc = apply_launch(s, best);
  if (rc != LBM_EHD_OK) return rc;
  if (std::any_of(own.begin(), own.end(), [](int b) { return b > 0; })) {
    double t_without = 0., t_with = 0.;
    rc = timed(&t_without);
    if (rc != LBM_EHD_OK) return rc;
    set_own(best, true);
    rc = apply_launch(s, best);
    if (rc != LBM_EHD_OK) return rc;
    rc = timed(&t_with);
    if (rc != LBM_EHD_OK) return rc;
    if (t_with >= t_without) {
      set_own(best, false);
      rc = apply_launch(s, best);
      if (rc != LBM_EHD_OK) return rc;
    }
  }
  // The knobs below change the schedule, not the tiles; their candidates
  // often time within a few per cent of each other, so a candidate replaces
  // the kept one only when it is faster by more than 2 % (the choice then
  // does not flip from run to run on timing noise).
  constexpr double KEEP = 0.98;
  // solo threshold: none, or the node count of one of the batch's lattice
  // sizes up to SOLO_CAP nodes (every instance of that size or smaller whose
  // loop stops on the successive change then runs in k_solo)
  constexpr long long SOLO_CAP = 192LL * 192LL;
  std::vector<long long> solo_c;
  for (const auto& p : s->params) {
    const long long n = (long long)p.nx * p.ny;
    if (n <= SOLO_CAP && p.pot_stop == LBM_EHD_STOP_CHANGE && std::find(solo_c.begin(), solo_c.end(), n) == solo_c.end())
      solo_c.push_back(n);
  }
  std::sort(solo_c.begin(), solo_c.end());
  auto try_shape = [&](const lbm_ehd_launch& L, double* t) {
    int r = apply_launch(s, L);
    if (r != LBM_EHD_OK) return r;
    return timed(t);
  };
  if (!solo_c.empty()) {
    best.solo_max_nodes = 0;
    rc = try_shape(best, &best_t);
    if (rc != LBM_EHD_OK) return rc;
    for (long long n : solo_c) {
      lbm_ehd_launch L = best;
      L.solo_max_nodes = (int32_t)n;
      double t = 0.;
      rc = try_shape(L, &t);
      if (rc != LBM_EHD_OK) return rc;
      if (t < KEEP * best_t) {
        best_t = t;
        best = L;
      }
    }
  }
  // With solo instances the longest loops left on the round path may be
  // shorter than the batch's: bands of their own again, from the round path's
  // own longest mean loop, kept only if they time faster.
  if (best.solo_max_nodes > 0) {
    double kmax_r = 0.;
    for (int i = 0; i < s->n_inst; ++i)
      if (!is_solo(best, s->params[i])) kmax_r = std::max(kmax_r, kbar[i]);
    std::vector<int> own_r(s->n_inst, 0);
    for (int i = 0; i < s->n_inst && kmax_r >= 2.; ++i) {
      if (is_solo(best, s->params[i])) continue;
      const double k = kbar[i] >= 2. ? kbar[i] / kmax_r : 0.;
      own_r[i] = k >= 0.8 ? 4 : (k >= 0.5 ? 8 : 0);
    }
    const std::vector<int> kept_bands = s->inst_band;
    own.swap(own_r);
    set_own(best, true);
    if (s->inst_band != kept_bands) {
      double t = 0.;
      rc = try_shape(best, &t);
      if (rc != LBM_EHD_OK) return rc;
      if (t < KEEP * best_t) {
        best_t = t;
      } else {
        s->inst_band = kept_bands;
        rc = apply_launch(s, best);
        if (rc != LBM_EHD_OK) return rc;
      }
    }
  }
  // rounds per captured chunk of the device loop: automatic, or fixed
  if (best.device_loop) {
    lbm_ehd_launch L0 = best;
    L0.rounds_per_graph = 0;
    rc = try_shape(L0, &best_t);
    if (rc != LBM_EHD_OK) return rc;
    best = L0;
    for (int rpg : {8, 32, 128}) {
      lbm_ehd_launch L = L0;
      L.rounds_per_graph = rpg;
      double t = 0.;
      rc = try_shape(L, &t);
      if (rc != LBM_EHD_OK) return rc;
      if (t < KEEP * best_t) {
        best_t = t;
        best = L;
      }
    }
  }
  // staggered start of half of the instances: off or on
  if (s->n_inst - s->n_solo > 1) {
    lbm_ehd_launch L0 = best;
    L0.stagger = 0;
    rc = try_shape(L0, &best_t);
    if (rc != LBM_EHD_OK) return rc;
    best = L0;
    lbm_ehd_launch L1 = L0;
    L1.stagger = 1;
    double t = 0.;
    rc = try_shape(L1, &t);
    if (rc != LBM_EHD_OK) return rc;
    if (t < KEEP * best_t) {
      best_t = t;
      best = L1;
    }
  }
  rc = apply_launch(s, best);
  if (rc != LBM_EHD_OK) return rc;
  if (out) *out = best;
  return refresh_status(s);
}

void lbm_ehd_destroy(lbm_ehd* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  delete s;
}

int lbm_ehd_timing(lbm_ehd* s, int32_t enable, lbm_ehd_timing_t* out) {
  if (!s || (enable != 0 && enable != 1)) return LBM_EHD_E_INVAL;
  HIP_OK(hipStreamSynchronize(s->stream));
  if (out) *out = s->tacc;
  if (enable) s->tacc = lbm_ehd_timing_t{};
  s->timing = enable != 0;
  return LBM_EHD_OK;
}

int lbm_ehd_abi_sizes(size_t* out, int32_t n) {
  const size_t sz[4] = {sizeof(lbm_ehd_params), sizeof(lbm_ehd_stats_t), sizeof(lbm_ehd_launch),
                        sizeof(lbm_ehd_timing_t)};
  if (!out || n < 0 || n > 4) return LBM_EHD_E_INVAL;
  for (int k = 0; k < n; ++k) out[k] = sz[k];
  return LBM_EHD_ABI_VERSION;
}

const char* lbm_ehd_strerror(int32_t code) {
  switch (code) {
    case LBM_EHD_OK: return "ok";
    case LBM_EHD_W_NOT_CONVERGED: return "an inner potential loop stopped at pot_max_iter";
    case LBM_EHD_W_DIVERGED: return "some instances diverged and were retired; the others continue";
    case LBM_EHD_E_INVAL: return "invalid argument";
    case LBM_EHD_E_WORKSPACE: return "workspace missing, too small or not 256-byte aligned";
    case LBM_EHD_E_HIP: return "HIP runtime error";
    case LBM_EHD_E_DIVERGED: return "non-finite state (diverged)";
    case LBM_EHD_E_STATE: return "handle in an unusable state";
    default: return "unknown status";
  }
}

}  // extern "C"
