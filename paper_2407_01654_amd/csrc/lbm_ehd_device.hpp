// Device side of the coupled two-phase EHD lattice Boltzmann step for gfx950.
//
// Layout in HBM (per instance, two pools: FP32 fields and the moving
// populations, FP32 or FP16).  A lattice row is cut into strips of 64
// columns (the last one padded to 64 slots).  Each pool stores, per row and
// strip, one block of 64 plane segments of 64 slots: element (plane p, row y,
// column x) sits at
//   y * ldx + (x / 64) * 4096 + p * 64 + x % 64,   ldx = 4096 * ceil(nx / 64).
// A 64-lane wave owns one strip: its stores cover whole aligned segments
// (256 bytes FP32, 128 bytes FP16) that no other wave writes, its loads reach
// into the neighbouring strips' segments (the columns left and right of the
// strip, which the stencils and the streaming need, are loaded by the wave
// itself), and the planes one pass touches lie together in each block
// (moving pool: g, l, f of both buffers in planes 0-47, h in 48-63; field
// pool: the 21 planes below in 0-20).
//   field pool : 13 auxiliary planes [psi, phi0, phi1, q0, q1, Fx, Fy, R, Gamma, Jx, Jy, refA, refB]
//                8 rest-population planes [buffer b][set s] (s = g, l, f, h)
//   moving pool: [buffer b][set g, l, f][direction 1..8], then [buffer b][direction 1..8] of h
// Every kernel pulls: the pre-collision population of direction i at x is the
// post-collision value of x - c_i held in the other buffer (half-way
// bounce-back / anti-bounce-back where x - c_i lies beyond a y wall).
//
// Stored values are deviations from a local reference known to both the
// writer and the reader, so that storage rounding acts on small numbers:
//   g_0 : minus phi of the previous step (phi plane b is the high part of the
//         g_0 stored in population buffer b)
//   l_i : (FP32 storage) minus w_i Q(node), Q the FP32 charge density the
//         writing node stored with it (q plane b belongs to population buffer
//         b); the reader adds w_i Q of the source node back, so the charge is
//         carried as the pair Q + (small remainder) and never rounded to FP32
//         as a whole between steps
//   h_i : minus k_i * psi_ref(node), k_0 = w_0 - 1, k_i = w_i, psi_ref the
//         potential at the start of the current outer step (planes refA/refB)
//   psi, refA, refB planes: minus the linear electrode profile
//         psi_lin(y) = psi_b + glin (y + 1/2), glin = (psi_t - psi_b) / ny,
//         whose isotropic-stencil gradient is exactly (0, glin)
//   FP16 moving populations additionally scale (pop - offset) / w_i.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// D2Q9 velocities (Eq. 37) and weights
constexpr int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
constexpr float W9[9] = {4.f / 9.f, 1.f / 9.f, 1.f / 9.f, 1.f / 9.f, 1.f / 9.f,
                         1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f};
constexpr float INVW[9] = {9.f / 4.f, 9.f, 9.f, 9.f, 9.f, 36.f, 36.f, 36.f, 36.f};
// potential equilibrium coefficients of Eq. (57): h_i^eq = KH[i] * psi
constexpr float KH[9] = {4.f / 9.f - 1.f, 1.f / 9.f, 1.f / 9.f, 1.f / 9.f, 1.f / 9.f,
                         1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f};
constexpr float CS2 = 1.f / 3.f;
constexpr float INV_CS2 = 3.f;
constexpr float INV_1MW0 = 9.f / 5.f;  // 1 / (1 - w_0)

enum { AUX_PSI = 0, AUX_PHI0, AUX_PHI1, AUX_Q0, AUX_Q1, AUX_FX, AUX_FY, AUX_R, AUX_GAM, AUX_JX, AUX_JY, AUX_REF0, AUX_REF1,
       N_AUX };
enum { SET_G = 0, SET_L = 1, SET_F = 2, SET_H = 3 };
enum { EN_CH = 1, EN_POT = 2, EN_NP = 4, EN_HYDRO = 8 };
constexpr int N_FPLANES = N_AUX + 8;   // aux + rest planes
constexpr int N_MPLANES = 64;          // moving planes
constexpr int BLOCK_PLANES = 64;       // plane segments per (row, strip) block of either pool
constexpr int SEG = 64;                // slots per plane segment
constexpr int HIST = 8192;             // K-history ring and replay capacity per instance

struct InstConst {
  long long off_f;   // element offset of the instance in the float pool
  long long off_m;   // element offset in the moving pool
  long long plane;   // elements between consecutive planes (one segment: 64)
  int nx, ny, ldx, walls;
  int enable, tile_begin, tile_end, owner_tile;
  float rho_v, drho, mu_v, dmu;
  float sig_v, dsig, eps_v, deps;      // deps = eps_v - eps_l
  float beta4, kappa, inv_tau_g, inv_tau_h;
  float inv_tau_l, fac_l, cs2_tau_h, conv_src;  // conv_src = 1 / (8 chi) (conventional potential scheme)
  float wet_b, wet_t, psi_b, psi_t;    // wet = sqrt(2 beta / kappa) cos(theta_eff)
  float glin, conv_k;                  // slope of the linear electrode profile (0 if periodic);
                                       // conv_k = 1 / (chi c_s^2)
  int q_impl;                          // 1: implicit charge closure of Eq. (66)
  int solo;                            // 1: advanced by a workgroup of its own (k_solo)
  int stagger;                         // 1: idles the first round of each stepping call
  int pad5;
  float scale[4], inv_scale[4];        // FP16 storage scale per set (powers of two)
  // the same folded with the weights of the moving directions, [set][0: w = 1/9, 1: w = 1/36]:
  // dec = w * inv_scale, enc = scale / w (exact: the scales are powers of two)
  float dec[4][2], enc[4][2];
  double tol;
  int max_iter, presolve_iters;
  int pot_stop;        // 1: the inner loop stops on the Poisson residual
  int pad2;
};

struct InstDyn {
  long long steps;
  long long total_iters;
  double last_r;
  double sum_phi, sum_q;
  int h_par;       // buffer holding the latest post-collision h
  int k;           // iterations of the running inner loop
  int active;      // inner loop running
  int target;      // forced iteration count of the running loop (0 = stop test)
  int status;      // bit0: hit pot_max_iter, bit1: non-finite
  int presolve_k;
  int replay_pos, replay_n;
  int ref_par;     // reference plane (refA/refB) the stored h are relative to
  int reref;       // next inner iteration re-references h to the other plane
  int phase;       // next round: 0 main pass, 1 inner iteration, 2 idle (staggered start)
  int presolve;    // 1 while the initial potential solve runs
  int s_done;      // outer steps finished in the running stepping call
  int n_target;    // outer steps requested by that call
  int bin;         // population buffer (and phi plane) holding the latest g, l, f
  int floor_stops; // inner loops that ended at the rounding floor of 16-bit h
  double last_res; // residual stop test: relative residual after the last iteration
};

struct Ctx {
  const InstConst* ic;
  InstDyn* dyn;
  const int4* tiles;       // (inst, x0, y0, y1)
  float* fpool;
  void* mpool;
  double2* part_main;      // per tile (sum phi, sum q)
  double2* part_pot;       // per tile (sum dpsi^2, sum psi^2)
  double* part_floor;      // per tile: sum of the dpsi^2 that rounding the stored h alone makes
  double2* part_res;       // per tile (sum r^2, sum s^2) of the Poisson residual
  int* khist;              // [n_inst][HIST]
  const int* replay;       // [n_inst][HIST]
  int* counters;           // [0] instances of the round path done with the running stepping call
  const int* solo_list;    // instances advanced by a workgroup of their own
  int n_inst, n_tiles;
  int n_ns_tiles;          // tiles of the round path: the work list's first n_ns_tiles entries
  int n_solo;
};

// ---------------------------------------------------------------------------
// HBM access through buffer resources: one descriptor per instance pool, the
// plane offset in the uniform soffset, the node offset (element offset of
// plane 0, 32 bits) in a VGPR.  Loads and stores outside a pool are discarded
// by the hardware range check.
// ---------------------------------------------------------------------------
constexpr unsigned BUF_DWORD3 = 0x00020000u;  // gfx9-family raw buffer descriptor word 3

struct Pools {
  __amdgpu_buffer_rsrc_t f;  // float pool of the instance (aux + rest planes)
  __amdgpu_buffer_rsrc_t m;  // moving pool of the instance
};

// Byte offsets of plane base + k at node byte offset nb, planes PS bytes
// apart (one segment: a compile-time stride).  A compile-time k goes into
// the vector offset, whose constant part the instruction's 12-bit immediate
// takes (k * PS < 4096 there); the run-time base, or a run-time k, into the
// scalar offset.  So the planes a wave touches need a scalar register per
// run-time base only, not one each.
template <unsigned PS>
__device__ __forceinline__ void plane_offsets(unsigned base, unsigned k, unsigned nb, unsigned& voff, unsigned& soff) {
  if (__builtin_constant_p(k) && k * PS < 4096u) {
    voff = nb + k * PS;
    soff = base * PS;
  } else {
    voff = nb;
    soff = (base + k) * PS;
  }
}
constexpr unsigned PF = (unsigned)SEG * 4u;  // bytes between float planes
// Cache policy of every store: non-temporal (the nt bit of the gfx940-family
// policy field).  A stored value is read again only in a later round, after
// the rest of the pass has streamed through L2; marking the stores as
// streaming leaves L2 to the loads that do reuse lines (halo rows and
// neighbour columns).
constexpr int ST_NT = 2;

template <class S>
__device__ __forceinline__ Pools make_pools(const Ctx& c, const InstConst& C) {
  Pools P;
  const unsigned n = (unsigned)C.ldx * (unsigned)C.ny;  // elements per pool
  P.f = __builtin_amdgcn_make_buffer_rsrc(c.fpool + C.off_f, 0, (int)(n * 4u), BUF_DWORD3);
  P.m = __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<typename S::T*>(c.mpool) + C.off_m, 0,
                                          (int)(n * (unsigned)sizeof(typename S::T)), BUF_DWORD3);
  return P;
}

// float plane pid at node index idx
__device__ __forceinline__ float fld(const Pools& P, int pid, unsigned idx) {
  unsigned vo, so;
  plane_offsets<PF>(0u, (unsigned)pid, idx * 4u, vo, so);
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(P.f, vo, so, 0));
}
__device__ __forceinline__ void fst(const Pools& P, int pid, unsigned idx, float v) {
  unsigned vo, so;
  plane_offsets<PF>(0u, (unsigned)pid, idx * 4u, vo, so);
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), P.f, vo, so, ST_NT);
}

// population storage: value = decode(stored) + offset
struct StoreF32 {
  using T = float;
  static constexpr bool kConvPot = false;
  static constexpr bool kChargeRef = true;  // l stored relative to w_i Q (see the layout notes)
  static constexpr bool kRound16 = false;   // stored values carry FP32 rounding only
  static constexpr unsigned PM = (unsigned)SEG * 4u;  // bytes between moving planes
  // moving plane mb + k (mb: first plane of a set and buffer)
  __device__ static float ld(const Pools& P, unsigned mb, unsigned k, unsigned idx, int, int, const InstConst&) {
    unsigned vo, so;
    plane_offsets<PM>(mb, k, idx * 4u, vo, so);
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(P.m, vo, so, 0));
  }
  __device__ static void st(const Pools& P, unsigned mb, unsigned k, unsigned idx, float v, int, int,
                            const InstConst&) {
    unsigned vo, so;
    plane_offsets<PM>(mb, k, idx * 4u, vo, so);
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), P.m, vo, so, ST_NT);
  }
};

struct StoreF16S {
  using T = __half;
  static constexpr bool kConvPot = false;
  // FP16 rounding (~5e-4) dwarfs the FP32 drift the charge reference removes:
  // l are stored relative to zero here
  static constexpr bool kChargeRef = false;
  static constexpr bool kRound16 = true;
  static constexpr unsigned PM = (unsigned)SEG * 2u;  // bytes between moving planes
  __device__ static float ld(const Pools& P, unsigned mb, unsigned k, unsigned idx, int i, int s,
                             const InstConst& C) {
    unsigned vo, so;
    plane_offsets<PM>(mb, k, idx * 2u, vo, so);
    const unsigned short b = __builtin_amdgcn_raw_buffer_load_b16(P.m, vo, so, 0);
    return (float)__builtin_bit_cast(_Float16, b) * C.dec[s][i >= 5];
  }
  // what a later load of v returns, minus v
  __device__ static float round_err(float v, int i, int s, const InstConst& C) {
    return __builtin_fmaf((float)(_Float16)(v * C.enc[s][i >= 5]), C.dec[s][i >= 5], -v);
  }
  __device__ static void st(const Pools& P, unsigned mb, unsigned k, unsigned idx, float v, int i, int s,
                            const InstConst& C) {
    const _Float16 h = (_Float16)(v * C.enc[s][i >= 5]);
    unsigned vo, so;
    plane_offsets<PM>(mb, k, idx * 2u, vo, so);
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, h), P.m, vo, so, ST_NT);
  }
};

// The conventional potential scheme (Sec. 3.3, the model the paper improves
// on) as a storage trait: the inner iteration relaxes every population with the
// local tau(x) = 1/2 + eps(phi) / (chi c_s^2) and drops the discrete forcing.
// Everything else is the storage type's.
template <class Base>
struct ConvPot : Base {
  static constexpr bool kConvPot = true;
};

// reciprocal from the hardware instruction (1 ulp): the collisions divide by
// local quantities (eps, rho, tau) that a correctly rounded division would
// cost ten instructions each for
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// periodic index for -n <= a < 2n
__device__ __forceinline__ int wrapi(int a, int n) {
  a = a < 0 ? a + n : a;
  return a >= n ? a - n : a;
}
// periodic index for any a
__device__ __forceinline__ int modi(int a, int n) {
  const int r = a % n;
  return r < 0 ? r + n : r;
}

constexpr int WAVE = 64;
constexpr int STRIP = WAVE;  // lattice columns per strip

// element offset of lattice column x (0 <= x < nx) in plane 0 of its row
__device__ __forceinline__ int col_slot(int x) { return (x / STRIP) * (BLOCK_PLANES * SEG) + (x % STRIP); }
// element offset of the strip starting at column x0 (a multiple of 64)
__device__ __forceinline__ int strip_base(int x0) { return (x0 / STRIP) * (BLOCK_PLANES * SEG); }

// slots of a column and of its periodic left and right neighbours
struct Cols {
  unsigned c, l, r;
};
__device__ __forceinline__ Cols cols_of(int x, int nx) {
  Cols k;
  k.c = (unsigned)col_slot(x);
  k.l = (unsigned)col_slot(wrapi(x - 1, nx));
  k.r = (unsigned)col_slot(wrapi(x + 1, nx));
  return k;
}

// one distribution set in one population buffer
template <class S>
struct PopView {
  Pools P;
  int rest_pid;   // float plane of the rest population
  unsigned mv0;   // moving plane of direction 1
  __device__ PopView(const Pools& pools, int buf, int set)
      : P(pools), rest_pid(N_AUX + buf * 4 + set),
        mv0((unsigned)(set < SET_H ? (buf * 3 + set) * 8 : 48 + buf * 8)) {}
  // stored value of direction i (the rest population as stored, which for g
  // is a deviation: no offset is added here, so that nothing waits on the load)
  __device__ float get(int i, unsigned idx, int set, const InstConst& C) const {
    return i == 0 ? fld(P, rest_pid, idx) : S::ld(P, mv0, (unsigned)(i - 1), idx, i, set, C);
  }
  // moving population stored in plane `dir` (wave-uniform, 1..8) decoded with
  // the weight of direction wi (opposite directions share their weight)
  __device__ float getm(int dir, unsigned idx, int wi, int set, const InstConst& C) const {
    return S::ld(P, mv0, (unsigned)(dir - 1), idx, wi, set, C);
  }
  __device__ void put(int i, unsigned idx, float v, int set, const InstConst& C, float off = 0.f) const {
    if (i == 0)
      fst(P, rest_pid, idx, v - off);
    else
      S::st(P, mv0, (unsigned)(i - 1), idx, v - off, i, set, C);
  }
};

// Pull of one set at node (x, y): pre-collision pop_i(x) = post_i(x - c_i),
// half-way bounce-back (post_{opp i}(x)) across a wall; the values as stored
// (the rest population of g is its deviation from the previous phi).  The
// wall case selects the plane and the address, so every direction is one
// load with no branch (all loads of a row can be in flight together).
template <class S>
__device__ __forceinline__ void pull_bb(const PopView<S>& v, const InstConst& C, int set, const Cols& k, int y,
                                        float out[9]) {
  const int ny = C.ny, ldx = C.ldx;
  const unsigned x = k.c, xl = k.l, xr = k.r;
  const bool wb = C.walls && y == 0, wt = C.walls && y == ny - 1;
  const int ydw = wrapi(y - 1, ny), yuw = wrapi(y + 1, ny);
  const unsigned row = (unsigned)(y * ldx), rd = (unsigned)(ydw * ldx), ru = (unsigned)(yuw * ldx);
  const unsigned me = row + x;
  out[0] = v.get(0, me, set, C);
  out[1] = v.getm(1, row + xl, 1, set, C);
  out[3] = v.getm(3, row + xr, 3, set, C);
  out[2] = v.getm(wb ? 4 : 2, wb ? me : rd + x, 2, set, C);
  out[5] = v.getm(wb ? 7 : 5, wb ? me : rd + xl, 5, set, C);
  out[6] = v.getm(wb ? 8 : 6, wb ? me : rd + xr, 6, set, C);
  out[4] = v.getm(wt ? 2 : 4, wt ? me : ru + x, 4, set, C);
  out[7] = v.getm(wt ? 5 : 7, wt ? me : ru + xr, 7, set, C);
  out[8] = v.getm(wt ? 6 : 8, wt ? me : ru + xl, 8, set, C);
}

// Pull of h in deviation form, in two parts so that the loads can be issued
// before the reference values are known.  Stored h are s_i = h_i - k_i
// psi_ref(node); load_h gathers the stored values the node pulls (its own
// post-collision opposite value across an electrode), dev_h turns them into
// delta_i = h_i(x) - k_i psi_ref(x), i.e. relative to the reference of the
// pulling node, with anti-bounce-back h_i = 2 w_i psi_wall - h*_{opp i}(x) at
// the electrodes.  ref[dy+1][dx+1] is psi_ref around (x, y).  All quantities
// stay small, so FP32 rounding acts on deviations, not on the potential.
template <class S>
__device__ __forceinline__ void load_h(const PopView<S>& v, const InstConst& C, const Cols& k, int y, float raw[9]) {
  pull_bb<S>(v, C, SET_H, k, y, raw);
}

__device__ __forceinline__ void dev_h(const InstConst& C, int y, const float raw[9], const float ref[3][3],
                                      float out[9]) {
#pragma clang fp contract(on)
  const bool wb = C.walls && y == 0, wt = C.walls && y == C.ny - 1;
  // ref holds psi_ref - psi_lin; sources one row below (c_y = +1) sit glin lower
  const float r0 = ref[1][1], gl = C.glin;
  const float bb = 2.f * (-0.5f * gl - r0), bt = 2.f * (0.5f * gl - r0);  // 2 (psi_wall - psi_ref(x))
  out[0] = raw[0];
  out[1] = raw[1] + KH[1] * (ref[1][0] - r0);
  out[3] = raw[3] + KH[3] * (ref[1][2] - r0);
  out[2] = wb ? W9[2] * bb - raw[2] : raw[2] + KH[2] * (ref[0][1] - r0 - gl);
  out[5] = wb ? W9[5] * bb - raw[5] : raw[5] + KH[5] * (ref[0][0] - r0 - gl);
  out[6] = wb ? W9[6] * bb - raw[6] : raw[6] + KH[6] * (ref[0][2] - r0 - gl);
  out[4] = wt ? W9[4] * bt - raw[4] : raw[4] + KH[4] * (ref[2][1] - r0 + gl);
  out[7] = wt ? W9[7] * bt - raw[7] : raw[7] + KH[7] * (ref[2][2] - r0 + gl);
  out[8] = wt ? W9[8] * bt - raw[8] : raw[8] + KH[8] * (ref[2][0] - r0 + gl);
}

// ---------------------------------------------------------------------------
// block reductions (fixed order: deterministic)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sums (a, b, c) over the block; result valid in every thread.  red: >= 3*16 doubles of LDS.
__device__ __forceinline__ double3 block_sum3(double a, double b, double c, double* red) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  __syncthreads();
  if (lane == 0) {
    red[3 * wv] = a;
    red[3 * wv + 1] = b;
    red[3 * wv + 2] = c;
  }
  __syncthreads();
  double3 r = make_double3(0.0, 0.0, 0.0);
  for (int w = 0; w < nw; ++w) {
    r.x += red[3 * w];
    r.y += red[3 * w + 1];
    r.z += red[3 * w + 2];
  }
  __syncthreads();
  return r;
}

// Sums (a, b) over the block; result valid in every thread.  red: >= 2*16 doubles of LDS.
__device__ __forceinline__ double2 block_sum2(double a, double b, double* red) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  a = wave_sum(a);
  b = wave_sum(b);
  __syncthreads();
  if (lane == 0) {
    red[2 * wv] = a;
    red[2 * wv + 1] = b;
  }
  __syncthreads();
  double2 r = make_double2(0.0, 0.0);
  for (int w = 0; w < nw; ++w) {
    r.x += red[2 * w];
    r.y += red[2 * w + 1];
  }
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------
// ghost values across the half-way walls (wetting Eq. 72; electrode potential)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float phi_ghost(float adj, float next, float wet) {
  float phw = fminf(fmaxf(0.5f * (3.f * adj - next), 0.f), 1.f);
  return adj + wet * (phw - phw * phw);
}

// ---------------------------------------------------------------------------
// wavefront-wide neighbour exchange: one 64-lane wave owns a strip of 64
// columns; lane t holds column x0 + t (and slot t of the strip's row
// segment).  The values of the neighbouring columns come from the
// neighbouring lanes via DPP wave shifts (no LDS, no barrier); at the strip's
// edges, from the halo value h the edge lane computed itself (lanes 0-31 hold
// the column left of the strip, lanes 32-63 the column right of it).
// ---------------------------------------------------------------------------

__device__ __forceinline__ float from_left(float v, float h) {   // lane t - 1; h in lane 0
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, h), __builtin_bit_cast(int, v),
                                                               0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_right(float v, float h) {  // lane t + 1; h in lane 63
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, h), __builtin_bit_cast(int, v),
                                                               0x130, 0xf, 0xf, false));
}

// Column of lane t in the strip starting at x0 with ncols lattice columns:
// x0 + t; the lanes beyond a narrow strip continue with the next two columns
// (periodically) and then repeat the second, so that the first of them, whose
// values stand in for the column right of the strip, sees its own right
// neighbour in the lane after it.  Only their loads reach other strips; their
// results go to padding.
__device__ __forceinline__ int lane_column(int x0, int ncols, int nx) {
  const int t = (int)(threadIdx.x & (WAVE - 1));
  return modi(x0 + min(t, ncols + 1), nx);
}
// Halo column of lane t: left of the wave's 64 columns for lanes 0-31, right
// of them for lanes 32-63 (lane 0 and lane 63 use it at the strip's edges).
__device__ __forceinline__ int halo_column(int x0, int nx) {
  const int t = (int)(threadIdx.x & (WAVE - 1));
  return modi(t < WAVE / 2 ? x0 - 1 : x0 + WAVE, nx);
}

// ---------------------------------------------------------------------------
// main pass of one tile: g, l, f (Algorithm 1 steps 2, 4, 5)
//   rows y0..y1-1 of the strip are advanced in order; each lane keeps the
//   order parameter (as the pair Phi + dphi) and the potential of rows y-1,
//   y, y+1 of its column in registers.  rnew: reference plane receiving psi^n
//   for the next inner loop.
// ---------------------------------------------------------------------------
template <class S>
__device__ void main_tile(const Ctx& c, const InstConst& C, int x0, int y0, int y1, int bin, int rnew,
                          double& acc_phi, double& acc_q) {
  const int t = threadIdx.x & (WAVE - 1);
  const int nx = C.nx, ny = C.ny, ldx = C.ldx;
  const int ncols = min(STRIP, nx - x0);
  const bool interior = t < ncols;
  const Cols cols = cols_of(lane_column(x0, ncols, nx), nx);
  const Cols hcols = cols_of(halo_column(x0, nx), nx);
  // every lane stores into its own slot of the strip's segment (the lanes
  // beyond a narrow strip into padding)
  const unsigned sslot = (unsigned)(strip_base(x0) + t);
  const Cols lcols = interior ? cols : Cols{sslot, sslot, sslot};
  const int en = C.enable;
  const Pools P = make_pools<S>(c, C);
  const int phi_in = AUX_PHI0 + bin, phi_out = AUX_PHI0 + (bin ^ 1);
  const int q_in = AUX_Q0 + bin, q_out = AUX_Q0 + (bin ^ 1);
  const PopView<S> gin(P, bin, SET_G), lin(P, bin, SET_L), fin(P, bin, SET_F);
  const PopView<S> gout(P, bin ^ 1, SET_G), lout(P, bin ^ 1, SET_L), fout(P, bin ^ 1, SET_F);

  // g of the row being advanced and of the next row; g[0] holds the stored
  // deviation d = g_0 - Phi with Phi = phi of the previous step.  phi = hi + lo
  // with hi = Phi (exact as stored) and lo = d + sum of the moving g.
  // The charge of the previous step, Q (FP32 as stored), of rows y-1, y, y+1
  // is kept the same way: the l of a node are decoded with Q of their source.
  // The same quantities of the halo column (suffix H) feed the edge lanes.
  float gcur[9], gnx[9];
  float hiM = 0.f, loM = 0.f, psM = 0.f, hi0 = 0.f, lo0 = 0.f, ps0 = 0.f, hiP = 0.f, loP = 0.f, psP = 0.f;
  float qM = 0.f, q0 = 0.f, qP = 0.f;
  float hiMH = 0.f, loMH = 0.f, psMH = 0.f, hi0H = 0.f, lo0H = 0.f, ps0H = 0.f, hiPH = 0.f, loPH = 0.f, psPH = 0.f;
  float qMH = 0.f, q0H = 0.f, qPH = 0.f;
  auto load_row = [&](int r, float* g, float& hi, float& lo, float& ps, float& qq, float& hiH, float& loH,
                      float& psH, float& qqH) {
    const int rw = wrapi(r, ny);
    float gh[9];
    pull_bb<S>(gin, C, SET_G, cols, rw, g);
    pull_bb<S>(gin, C, SET_G, hcols, rw, gh);
    const unsigned o = (unsigned)(rw * ldx) + cols.c, oh = (unsigned)(rw * ldx) + hcols.c;
    hi = fld(P, phi_in, o);
    hiH = fld(P, phi_in, oh);
    ps = fld(P, AUX_PSI, o);
    psH = fld(P, AUX_PSI, oh);
    if constexpr (S::kChargeRef) {
      qq = fld(P, q_in, o);
      qqH = fld(P, q_in, oh);
    }
    float d = g[0], dh = gh[0];
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      d += g[i];
      dh += gh[i];
    }
    lo = d;
    loH = dh;
  };
  // (above the bottom electrode the row below is replaced by ghosts)
  load_row((C.walls && y0 == 0) ? y0 : y0 - 1, gnx, hiM, loM, psM, qM, hiMH, loMH, psMH, qMH);
  load_row(y0, gcur, hi0, lo0, ps0, q0, hi0H, lo0H, ps0H, q0H);

  for (int y = y0; y < y1; ++y) {
    const bool top_wall = C.walls && y + 1 == ny;
    const bool bot_wall = C.walls && y == 0;
    // every load of the row is issued before the first use of any of them:
    // l, f and the lagged fields of row y, then g, Phi and psi of row y + 1
    // and of the halo column (the lanes beyond a narrow strip, whose
    // collision results land in padding, read l, f and the lagged fields from
    // their own slots: no line of another strip is touched for them)
    const unsigned sidx = (unsigned)(y * ldx) + sslot, idx = interior ? (unsigned)(y * ldx) + cols.c : sidx;
    float l[9], f[9];
    pull_bb<S>(lin, C, SET_L, lcols, y, l);
    pull_bb<S>(fin, C, SET_F, lcols, y, f);
    // the lagged closure of Eq. (66) reads R^{n-1}; the implicit one needs none
    const float R_prev = C.q_impl ? 0.f : fld(P, AUX_R, idx);
    const float Fx_prev = fld(P, AUX_FX, idx), Fy_prev = fld(P, AUX_FY, idx);
    const float G_prev = fld(P, AUX_GAM, idx);
    const float Jx_prev = fld(P, AUX_JX, idx), Jy_prev = fld(P, AUX_JY, idx);
    // below the top electrode the row above is replaced by ghosts
    load_row(top_wall ? y : y + 1, gnx, hiP, loP, psP, qP, hiPH, loPH, psPH, qPH);
    // ghost rows across the walls, per column: wetting Eq. (72) for phi (kept
    // in the low part), psi_ghost = 2 psi_wall - psi_adj (psi is stored minus
    // the linear electrode profile, which passes through psi_wall)
    if (bot_wall) {
      const float a = hi0 + lo0, aH = hi0H + lo0H;
      hiM = hi0;
      loM = lo0 + (phi_ghost(a, hiP + loP, C.wet_b) - a);
      psM = -ps0;
      hiMH = hi0H;
      loMH = lo0H + (phi_ghost(aH, hiPH + loPH, C.wet_b) - aH);
      psMH = -ps0H;
    }
    if (top_wall) {
      const float a = hi0 + lo0, aH = hi0H + lo0H;
      hiP = hi0;
      loP = lo0 + (phi_ghost(a, hiM + loM, C.wet_t) - a);
      psP = -ps0;
      hiPH = hi0H;
      loPH = lo0H + (phi_ghost(aH, hiMH + loMH, C.wet_t) - aH);
      psPH = -ps0H;
    }
    // 3 x 3 neighbourhoods [dy+1][dx+1] from the neighbouring lanes
    float hh[3][3], lo[3][3], ps[3][3];
    const float hhH[3] = {hiMH, hi0H, hiPH}, loH[3] = {loMH, lo0H, loPH}, psH[3] = {psMH, ps0H, psPH};
    hh[0][1] = hiM; lo[0][1] = loM; ps[0][1] = psM;
    hh[1][1] = hi0; lo[1][1] = lo0; ps[1][1] = ps0;
    hh[2][1] = hiP; lo[2][1] = loP; ps[2][1] = psP;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      hh[d][0] = from_left(hh[d][1], hhH[d]);
      hh[d][2] = from_right(hh[d][1], hhH[d]);
      lo[d][0] = from_left(lo[d][1], loH[d]);
      lo[d][2] = from_right(lo[d][1], loH[d]);
      ps[d][0] = from_left(ps[d][1], psH[d]);
      ps[d][2] = from_right(ps[d][1], psH[d]);
    }
    // Q of the source node of each pulled l_i minus Q of this node (the
    // node itself across a wall, where l_i is its own bounced value)
    float dq[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if constexpr (S::kChargeRef) {
      const float qlM = from_left(qM, qMH), qrM = from_right(qM, qMH), ql0 = from_left(q0, q0H);
      const float qr0 = from_right(q0, q0H), qlP = from_left(qP, qPH), qrP = from_right(qP, qPH);
      dq[0] = 0.f;
      dq[1] = ql0 - q0;
      dq[3] = qr0 - q0;
      dq[2] = bot_wall ? 0.f : qM - q0;
      dq[5] = bot_wall ? 0.f : qlM - q0;
      dq[6] = bot_wall ? 0.f : qrM - q0;
      dq[4] = top_wall ? 0.f : qP - q0;
      dq[7] = top_wall ? 0.f : qrP - q0;
      dq[8] = top_wall ? 0.f : qlP - q0;
    }
    {  // every lane: the results of lanes beyond a narrow strip land in padding slots
      // isotropic gradient and Laplacian (Sec. 3.2) on differences from the
      // centre node (sum_i w_i c_i = 0), hi and lo parts separately
      float gphx = 0.f, gphy = 0.f, lap = 0.f, gpsx = 0.f, gpsy = 0.f;
      const float hc = hh[1][1], lc = lo[1][1];
      const float phi = hc + lc;
#pragma unroll
      for (int i = 1; i < 9; ++i) {
        const float dphi = (hh[1 + CY[i]][1 + CX[i]] - hc) + (lo[1 + CY[i]][1 + CX[i]] - lc);
        const float b = ps[1 + CY[i]][1 + CX[i]];
        gphx += W9[i] * CX[i] * dphi;
        gphy += W9[i] * CY[i] * dphi;
        lap += 2.f * W9[i] * dphi;
        gpsx += W9[i] * CX[i] * b;
        gpsy += W9[i] * CY[i] * b;
      }
      gphx *= INV_CS2;
      gphy *= INV_CS2;
      lap *= INV_CS2;
      // E = -grad psi = -(grad of the deviation + (0, glin)), Eq. (32)
      const float Ex = -gpsx * INV_CS2, Ey = -gpsy * INV_CS2 - C.glin;


      const float rho = C.rho_v + phi * C.drho;
      const float grx = C.drho * gphx, gry = C.drho * gphy;
      const float eps = C.eps_v + phi * phi * (2.f * phi - 3.f) * C.deps;
      const float deps = 6.f * phi * (phi - 1.f) * C.deps;
      const float sig = C.sig_v + phi * C.dsig;
      const float gE = gphx * Ex + gphy * Ey;
      // R = -(sigma / eps) q + B, Eq. (61)
      const float se = sig * rcp(eps);
      const float B = se * deps * gE - C.dsig * gE;
      // q^n = Q + lo_q, Eq. (66): d_i = l_i - w_i Q(this node) (without the
      // charge reference Q = 0 and d_i = l_i); lagged: R^{n-1} / 2 added;
      // implicit: q = (Q + sum d + B/2) / (1 + sigma / (2 eps))
      float dl[9], lo_q = 0.f;
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        dl[i] = l[i] + W9[i] * dq[i];
        lo_q += dl[i];
      }
      if (C.q_impl) {
        const float hk = 0.5f * se;
        lo_q = (lo_q + 0.5f * B - q0 * hk) * rcp(1.f + hk);
      } else {
        lo_q += 0.5f * R_prev;
      }
      const float q = q0 + lo_q;
      float ux = 0.f, uy = 0.f;
      if (en & EN_HYDRO) {
        float mx = 0.f, my = 0.f;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
          mx += CX[i] * f[i];
          my += CY[i] * f[i];
        }
        const float ir = rcp(rho);
        ux = (mx + 0.5f * Fx_prev) * ir;                    // Eq. (43), lagged F
        uy = (my + 0.5f * Fy_prev) * ir;
      }
      const float uu = ux * ux + uy * uy;
      const float ugr = ux * grx + uy * gry;
      float sumf = 0.f;
#pragma unroll
      for (int i = 1; i < 9; ++i) sumf += f[i];
      const float s0 = -W9[0] * uu * (0.5f * INV_CS2);
      const float p = CS2 * INV_1MW0 * (sumf + 0.5f * ugr + rho * s0);   // Eq. (44)
      const float EE = Ex * Ex + Ey * Ey;
      const float mu_c = C.beta4 * phi * (phi - 0.5f) * (phi - 1.f) - C.kappa * lap - 0.5f * deps * EE;  // Eq. (31)
      const float Fx = mu_c * gphx + q * Ex, Fy = mu_c * gphy + q * Ey;                                 // Eq. (30)
      const float R = -se * q + B;                                                                     // Eq. (57)
      const float Gam = ux * gphx + uy * gphy;
      const float Jx = q * ux, Jy = q * uy;

      if (en & EN_CH) {  // Eq. (45)-(47)
        const float tg = C.inv_tau_g;
        const float dG = Gam + 0.5f * (Gam - G_prev);
        // rest population as deviation from the phi written now, phi = fl(Phi + lc):
        // g_0 - g_0^eq = (d - lc) + (1 - w_0) mu_c with the exact order parameter
        // Phi + lc, and the stored value relative to phi starts from d - (phi - Phi),
        // which keeps the rounding of the sum Phi + lc (phi - Phi is exact: both
        // lie within a factor two of each other) instead of dropping it each step
        const float dd = gcur[0] - lc;
        const float dstore = gcur[0] - (phi - hc);
        const float coef0 = W9[0] * (-1.f + (0.f - 2.f * CS2) * (0.5f * INV_CS2));
        gout.put(0, sidx, dstore - (dd + (1.f - W9[0]) * mu_c) * tg + coef0 * dG, SET_G, C);
#pragma unroll
        for (int i = 1; i < 9; ++i) {
          const float geq = W9[i] * mu_c;
          const float coef = W9[i] * (-1.f + ((float)(CX[i] * CX[i] + CY[i] * CY[i]) - 2.f * CS2) * (0.5f * INV_CS2));
          gout.put(i, sidx, gcur[i] - (gcur[i] - geq) * tg + coef * dG, SET_G, C);
        }
        fst(P, phi_out, sidx, phi);
      }
      if (en & EN_NP) {  // Eq. (62)-(65) on deviations
        // stored: l*_i - w_i Qn, Qn = fl(q) written below; with dQ = Qn - Q,
        // l_i - w_i Qn = d_i - w_i dQ and l_i - l_i^eq = d_i - w_i (lo_q + q c_i.u / c_s^2)
        const float tl = C.inv_tau_l, fl = C.fac_l;
        const float dJx = Jx - Jx_prev, dJy = Jy - Jy_prev;
        const float dQ = S::kChargeRef ? q - q0 : 0.f;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
          const float cu = CX[i] * ux + CY[i] * uy;
          const float neq = dl[i] - W9[i] * (lo_q + q * cu * INV_CS2);
          const float src = fl * W9[i] * (R + (CX[i] * dJx + CY[i] * dJy) * INV_CS2);
          lout.put(i, sidx, (dl[i] - W9[i] * dQ) - neq * tl + src, SET_L, C);
        }
      }
      if (en & EN_HYDRO) {  // Eq. (38)-(42)
        const float mu = C.mu_v + phi * C.dmu;
        const float tau_f = 0.5f + mu * rcp(rho) * INV_CS2;
        const float itf = rcp(tau_f), ff = 1.f - 0.5f * itf;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
          const float cu = CX[i] * ux + CY[i] * uy;
          const float si = W9[i] * (cu * INV_CS2 + cu * cu * (0.5f * INV_CS2 * INV_CS2) - uu * (0.5f * INV_CS2));
          const float feq = (i == 0 ? (W9[0] - 1.f) : W9[i]) * p * INV_CS2 + rho * si;
          const float cg = CX[i] * grx + CY[i] * gry;
          const float rb = W9[i] * (ugr + (CX[i] * Fx + CY[i] * Fy) * INV_CS2 + (cu * cg - CS2 * ugr) * INV_CS2);
          fout.put(i, sidx, f[i] - (f[i] - feq) * itf + ff * rb, SET_F, C);
        }
      }
      // without the Nernst-Planck set the l stay as initialised, and so does
      // the reference they were stored against
      fst(P, q_out, sidx, (!S::kChargeRef || (en & EN_NP)) ? q : q0);
      fst(P, AUX_FX, sidx, Fx);
      fst(P, AUX_FY, sidx, Fy);
      if (!C.q_impl) fst(P, AUX_R, sidx, R);
      fst(P, AUX_GAM, sidx, Gam);
      fst(P, AUX_JX, sidx, Jx);
      fst(P, AUX_JY, sidx, Jy);
      fst(P, AUX_REF0 + rnew, sidx, ps0);   // psi^n: reference of the next inner loop
      if (interior) {
        acc_phi += (double)phi;
        acc_q += (double)q0 + (double)lo_q;
      }
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) gcur[i] = gnx[i];
    hiM = hi0; loM = lo0; psM = ps0; qM = q0;
    hi0 = hiP; lo0 = loP; ps0 = psP; q0 = qP;
    hiMH = hi0H; loMH = lo0H; psMH = ps0H; qMH = q0H;
    hi0H = hiPH; lo0H = loPH; ps0H = psPH; q0H = qPH;
  }
}

// ---------------------------------------------------------------------------
// one inner iteration of the potential set on one tile (Algorithm 1 step 3)
//   every lane collides its node of each row, and also the node of its halo
//   column (left of the strip for lanes 0-31, right of it for 32-63), whose
//   post-collision values stream into the strip's edge columns.  The
//   arithmetic runs on deviations from psi_ref (plane rdec): with delta_i =
//   h_i - k_i psi_ref, psi = psi_ref + sum delta_i / (1 - w_0) and h_i -
//   h_i^eq = delta_i - k_i (psi - psi_ref).  Each post-collision moving
//   population is also expressed relative to the reference of the node it
//   streams to, so the row behind gathers its streamed potential psi^(k) (and
//   the stop-test sums) from the neighbouring lanes' registers without
//   further references.  renc: plane the stored h are made relative to
//   (differs from rdec on the iteration that moves h to a fresh reference);
//   capture: also write psi^(k) into the spare reference plane for such a move.
// ---------------------------------------------------------------------------
template <class S>
__device__ void pot_tile(const Ctx& c, const InstConst& C, int x0, int y0, int y1, int hin, int phip,
                         int rdec, int renc, int capture, double& acc_num, double& acc_den,
                         double& acc_floor) {
  // Multiply-adds are fused as the expressions are written, never across
  // them: the rows of a band alternate between two copies of the row code,
  // and with free fusion the two copies could round differently, so that
  // results would depend on where the bands start.
#pragma clang fp contract(on)
  const int t = threadIdx.x & (WAVE - 1);
  const int nx = C.nx, ny = C.ny, ldx = C.ldx;
  const int ncols = min(STRIP, nx - x0);
  const bool interior = t < ncols;
  const Cols cols = cols_of(lane_column(x0, ncols, nx), nx);
  // halo node of the lane; its neighbour towards the strip is the edge lane's
  // own column, the one away from it (xo) is loaded
  const bool left = t < WAVE / 2;
  const Cols hcols = cols_of(halo_column(x0, nx), nx);
  const unsigned xo = (unsigned)col_slot(modi(left ? x0 - 2 : x0 + WAVE + 1, nx));
  const unsigned sslot = (unsigned)(strip_base(x0) + t);  // own slot of the strip's segment
  const Pools P = make_pools<S>(c, C);
  const PopView<S> hv(P, hin, SET_H), hout(P, hin ^ 1, SET_H);
  const int phi_pid = AUX_PHI0 + phip, q_pid = AUX_Q0 + phip, rdec_pid = AUX_REF0 + rdec, renc_pid = AUX_REF0 + renc;
  const int cap_pid = AUX_REF0 + (rdec ^ 1);
  const float gl = C.glin;

  // reference psi_ref - psi_lin of rows r-1, r, r+1: own column, halo
  // column, and the halo's outer neighbour
  float Rc[3] = {0.f, 0.f, 0.f}, Rh[3] = {0.f, 0.f, 0.f}, Ro[3] = {0.f, 0.f, 0.f};
  // raw loads of a reference row (rows beyond an electrode read the wall row
  // and are zeroed in set_ref: they only feed values that the walls replace)
  struct RefRaw {
    float own, h, o;
  };
  auto load_ref = [&](int r) {
    const int rr = C.walls ? min(max(r, 0), ny - 1) : modi(r, ny);  // r may reach -2 and ny + 1
    const unsigned row = (unsigned)(rr * ldx);
    RefRaw q;
    q.own = fld(P, rdec_pid, row + cols.c);
    q.h = fld(P, rdec_pid, row + hcols.c);
    q.o = fld(P, rdec_pid, row + xo);
    return q;
  };
  auto set_ref = [&](int r, const RefRaw& q, int k) {
    const bool zero = C.walls && (r < 0 || r >= ny);
    Rc[k] = zero ? 0.f : q.own;
    Rh[k] = zero ? 0.f : q.h;
    Ro[k] = zero ? 0.f : q.o;
  };

  // post-collision deviations ts_i = h*_i - k_i psi_ref(x) of a node (Eq. 56);
  // returns psi - psi_ref (Eq. 58)
  auto collide = [&](int rw, const float raw[9], const float ref[3][3], float phi, float q, float ts[9]) {
    float dl[9];
    dev_h(C, rw, raw, ref, dl);
    float dpsi = 0.f;
#pragma unroll
    for (int i = 1; i < 9; ++i) dpsi += dl[i];
    dpsi *= INV_1MW0;                                         // Eq. (58), minus psi_ref
    const float eh = phi * phi * (2.f * phi - 3.f) * C.deps;  // eps_hat of Eq. (55)
    if constexpr (S::kConvPot) {
      // conventional scheme: eps(phi) = eps_v + eps_hat = chi c_s^2 (tau - 1/2)
      const float itau = rcp(0.5f + (C.eps_v + eh) * C.conv_k);
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const float src = i == 0 ? 0.f : C.conv_src * q;
        ts[i] = dl[i] - (dl[i] - KH[i] * dpsi) * itau + src;
      }
    } else {
      float mx = 0.f, my = 0.f;
#pragma unroll
      for (int i = 1; i < 9; ++i) {
        mx += CX[i] * dl[i];
        my += CY[i] * dl[i];
      }
      const float id = -rcp(eh + C.cs2_tau_h);                  // Eq. (59)
      const float gpx = mx * id, gpy = my * id;
      const float fk = eh * INV_CS2 * C.inv_tau_h;
      // h*_i = (1 - 1/tau) d_i + k_i psi' / tau - fk w_i c_i . grad psi + src_i,
      // psi' = dpsi, with c_i . grad psi formed once per direction pair
      const float a = 1.f - C.inv_tau_h, bdp = dpsi * C.inv_tau_h, src = 0.125f * q;
      const float base1 = __builtin_fmaf(KH[1], bdp, src), base5 = __builtin_fmaf(KH[5], bdp, src);
      const float c1 = fk * W9[1], c5 = fk * W9[5];
      const float d1 = gpx + gpy, d2 = gpy - gpx;
      const float g[9] = {0.f, gpx, gpy, -gpx, -gpy, d1, d2, -d1, -d2};
      ts[0] = __builtin_fmaf(a, dl[0], KH[0] * bdp);
#pragma unroll
      for (int i = 1; i < 9; ++i)
        ts[i] = __builtin_fmaf(a, dl[i], __builtin_fmaf(-(i < 5 ? c1 : c5), g[i], i < 5 ? base1 : base5));
    }
    return dpsi;
  };
  // The halo node's post-collision values that stream into the edge column,
  // relative to the edge node's reference: directions 1, 5, 8 from the left
  // halo, 3, 6, 7 from the right one (c_x = +1 or -1 and c_y = 0, +1, -1).
  // Only the edge lanes use them, so only these three are formed, with the
  // direction picked per lane; per direction the arithmetic is the
  // collision's above, term for term.  ref: the halo node's neighbourhood,
  // whose column 1 + c_x is the edge column (Rc of the edge lane).
  const float sx = left ? 1.f : -1.f;
  auto collide_edge = [&](int rw, const float raw[9], const float ref[3][3], float phi, float q, float& hA,
                          float& hB, float& hC) {
    float dl[9];
    dev_h(C, rw, raw, ref, dl);
    float dpsi = 0.f;
#pragma unroll
    for (int i = 1; i < 9; ++i) dpsi += dl[i];
    dpsi *= INV_1MW0;
    const float eh = phi * phi * (2.f * phi - 3.f) * C.deps;
    const float dA = left ? dl[1] : dl[3], dB = left ? dl[5] : dl[6], dC = left ? dl[8] : dl[7];
    float tA, tB, tC;
    if constexpr (S::kConvPot) {
      const float itau = rcp(0.5f + (C.eps_v + eh) * C.conv_k);
      const float src = C.conv_src * q;
      tA = dA - (dA - KH[1] * dpsi) * itau + src;
      tB = dB - (dB - KH[5] * dpsi) * itau + src;
      tC = dC - (dC - KH[8] * dpsi) * itau + src;
    } else {
      float mx = 0.f, my = 0.f;
#pragma unroll
      for (int i = 1; i < 9; ++i) {
        mx += CX[i] * dl[i];
        my += CY[i] * dl[i];
      }
      const float id = -rcp(eh + C.cs2_tau_h);
      const float gpx = mx * id, gpy = my * id;
      const float fk = eh * INV_CS2 * C.inv_tau_h;
      const float a = 1.f - C.inv_tau_h, bdp = dpsi * C.inv_tau_h, src = 0.125f * q;
      const float base1 = __builtin_fmaf(KH[1], bdp, src), base5 = __builtin_fmaf(KH[5], bdp, src);
      const float c1 = fk * W9[1], c5 = fk * W9[5];
      // c . grad psi of the lane's three directions: sx gpx, sx gpx + gpy, sx gpx - gpy (the
      // products with sx = +-1 are exact, so these equal the own collision's values)
      const float gA = sx * gpx, gB = __builtin_fmaf(sx, gpx, gpy), gC = __builtin_fmaf(sx, gpx, -gpy);
      tA = __builtin_fmaf(a, dA, __builtin_fmaf(-c1, gA, base1));
      tB = __builtin_fmaf(a, dB, __builtin_fmaf(-c5, gB, base5));
      tC = __builtin_fmaf(a, dC, __builtin_fmaf(-c5, gC, base5));
    }
    const float r0 = ref[1][1];
    hA = tA + KH[1] * (r0 - Rc[1]);
    hB = tB + KH[5] * (r0 - Rc[2] - gl);
    hC = tC + KH[8] * (r0 - Rc[0] + gl);
  };

  // moving post-collision values of the rows behind, relative to the
  // reference of their destination node
  // (directions 1, 3 from the row behind; 2, 5, 6 from two rows behind)
  float u1p = 0.f, u3p = 0.f, u2p = 0.f, u5p = 0.f, u6p = 0.f, u2pp = 0.f, u5pp = 0.f, u6pp = 0.f;
  // the same from the halo node into the edge column: direction 1 (left
  // halo) or 3 (right) of the row behind, 5 or 6 of two rows behind
  float hAp = 0.f, hBp = 0.f, hBpp = 0.f;
  // own post-collision values of the row behind relative to its own reference (walls)
  float w2p = 0.f, w4p = 0.f, w5p = 0.f, w6p = 0.f, w7p = 0.f, w8p = 0.f, r0p = 0.f, dcp = 0.f;

  // streamed potential of row rf (relative to its reference), rf = row behind
  auto finish_row = [&](int rf, float u4, float u7, float u8, float hC, double& num, double& den) {
    const bool wb = C.walls && rf == 0, wt = C.walls && rf == ny - 1;
    const float u7r = from_right(u7, hC), u8l = from_left(u8, hC);
    const float u1l = from_left(u1p, hAp), u3r = from_right(u3p, hAp);
    const float u5l = from_left(u5pp, hBpp), u6r = from_right(u6pp, hBpp);
    if (rf < 0) return;
    const float bb = 2.f * (-0.5f * gl - r0p), bt = 2.f * (0.5f * gl - r0p);  // 2 (psi_wall - psi_ref)
    float a = u1l + u3r;
    a += wb ? W9[2] * bb - w4p : u2pp;
    a += wb ? W9[5] * bb - w7p : u5l;
    a += wb ? W9[6] * bb - w8p : u6r;
    a += wt ? W9[4] * bt - w2p : u4;
    a += wt ? W9[7] * bt - w5p : u7r;
    a += wt ? W9[8] * bt - w6p : u8l;
    const float dnew = a * INV_1MW0;
    const unsigned o = (unsigned)(wrapi(rf, ny) * ldx) + sslot;
    const float pn = r0p + dnew;  // psi^(k) - psi_lin
    fst(P, AUX_PSI, o, pn);
    if (capture) fst(P, cap_pid, o, pn);
    if (!interior) return;
    const double d = (double)dnew - (double)dcp;
    const double pc = (double)C.psi_b + (double)gl * ((double)wrapi(rf, ny) + 0.5) + (double)r0p + (double)dcp;
    num += d * d;
    den += pc * pc;
  };

  const int rs = (C.walls && y0 == 0) ? 0 : y0 - 1;
  const int re = (C.walls && y1 == ny) ? ny - 1 : y1;
  set_ref(rs - 1, load_ref(rs - 1), 0);
  set_ref(rs, load_ref(rs), 1);
  // Every load of a row is issued one row ahead: h pulled into the row at the
  // own and the halo column, phi and q there, the stored reference of a
  // re-reference, and the reference row after it.  The loads of row r + 1 are
  // in flight while row r is collided, so each wave keeps two rows of loads
  // outstanding.
  struct RowIn {
    float raw[9], rawH[9], phi, q, phiH, qH, renc;
    RefRaw ref;
  };
  auto fetch = [&](int r) {
    RowIn in;
    const int rw = wrapi(r, ny);
    const unsigned row = (unsigned)(rw * ldx);
    const unsigned idx = row + cols.c, hidx = row + hcols.c;
    load_h<S>(hv, C, cols, rw, in.raw);
    load_h<S>(hv, C, hcols, rw, in.rawH);
    in.phi = fld(P, phi_pid, idx);
    in.q = fld(P, q_pid, idx);
    in.phiH = fld(P, phi_pid, hidx);
    in.qH = fld(P, q_pid, hidx);
    in.renc = fld(P, renc_pid, row + sslot);  // only stores use it
    in.ref = load_ref(r + 1);
    return in;
  };
  auto row = [&](int r, const RowIn& cur) {
    const int rw = wrapi(r, ny);
    const unsigned sidx = (unsigned)(rw * ldx) + sslot;
    const float* raw = cur.raw;
    const float* rawH = cur.rawH;
    const float phi = cur.phi, q = cur.q, phiH = cur.phiH, qH = cur.qH, renc_v = cur.renc;
    set_ref(r + 1, cur.ref, 2);
    // 3 x 3 reference neighbourhoods of the own node and of the halo node
    float ref[3][3], refH[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      ref[k][0] = from_left(Rc[k], Rh[k]);
      ref[k][1] = Rc[k];
      ref[k][2] = from_right(Rc[k], Rh[k]);
      refH[k][0] = left ? Ro[k] : Rc[k];
      refH[k][1] = Rh[k];
      refH[k][2] = left ? Rc[k] : Ro[k];
    }
    float ts[9];
    const float dpsi = collide(rw, raw, ref, phi, q, ts);
    float hA, hB, hC;
    collide_edge(rw, rawH, refH, phiH, qH, hA, hB, hC);
    {
      const bool store = r >= y0 && r < y1;  // rows of the band (all lanes)
      const float shift = (store && renc != rdec) ? ref[1][1] - renc_v : 0.f;
      if (store) {
        float e2 = 0.f;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
          const float v = ts[i] + KH[i] * shift;
          hout.put(i, sidx, v, SET_H, C);
          if constexpr (S::kRound16) {
            // what 16-bit storage adds to the moving values (the rest one is FP32)
            if (i > 0) {
              const float e = S::round_err(v, i, SET_H, C);
              e2 += e * e;
            }
          }
        }
        if (S::kRound16 && interior) acc_floor += (double)(e2 * (INV_1MW0 * INV_1MW0));
      }
    }
    // relative to the destination's reference: h*_i - k_i psi_ref(x + c_i)
    //   psi_ref(x) - psi_ref(x + c_i) = ref(centre) - ref(x + c_i) - c_iy glin
    float u[9];
#pragma unroll
    for (int i = 1; i < 9; ++i) u[i] = ts[i] + KH[i] * (ref[1][1] - ref[1 + CY[i]][1 + CX[i]] - (float)CY[i] * gl);
    // gather the row behind (r - 1) now that row r is known
    finish_row(r - 1 >= y0 && r - 1 < y1 ? r - 1 : -1, u[4], u[7], u[8], hC, acc_num, acc_den);
    // roll the row state
    u2pp = u2p; u5pp = u5p; u6pp = u6p;
    u2p = u[2]; u5p = u[5]; u6p = u[6];
    u1p = u[1]; u3p = u[3];
    hBpp = hBp; hBp = hB; hAp = hA;
    w2p = ts[2]; w4p = ts[4]; w5p = ts[5]; w6p = ts[6]; w7p = ts[7]; w8p = ts[8];
    r0p = ref[1][1];
    dcp = dpsi;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      Rc[k] = Rc[k + 1];
      Rh[k] = Rh[k + 1];
      Ro[k] = Ro[k + 1];
    }
  };
  // two rows per trip with two row buffers taking turns, so that no copy
  // carries the fetched values from one row to the next.  The fetch of the
  // next row is unconditional, so that the waits for this row's values stay
  // ahead of the next row's loads (the last row fetches itself again: cache
  // hits).
  RowIn bufA = fetch(rs);
  for (int r = rs; r <= re; r += 2) {
    const RowIn bufB = fetch(min(r + 1, re));
    row(r, bufA);
    if (r + 1 > re) break;
    bufA = fetch(min(r + 2, re));
    row(r + 1, bufB);
  }
  // the top row of a band ending at the top wall has no row above: gather it
  // from its own anti-bounce-back values
  if (C.walls && y1 == ny) finish_row(ny - 1, 0.f, 0.f, 0.f, 0.f, acc_num, acc_den);
}

}  // namespace lbm
