// qed_device.h -- device-side building blocks of the QED step for gfx950 (CDNA4).
//
// Internal header of libqed.  Everything here is __device__ code written for 64-lane
// wavefronts; the host entry points live in qed_api.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qed.h"

namespace qedk {

constexpr double kAlpha = 7.2973525693e-3;  // fine-structure constant, CODATA 2018
constexpr double kPi = 3.141592653589793238;
constexpr double kInvSqrt3Pi = 0.18377629847393068;  // 1 / (sqrt(3) pi)
constexpr int kTableN = QED_TABLE_N;
constexpr double kLog2ZLo = -20.0;  // first node z = 2^-20
constexpr double kLog2ZHi = 7.0;    // last node z = 2^7; functions vanish beyond
constexpr double kZLo = 0x1p-20;
constexpr double kZHi = 128.0;
constexpr double kNodesPerLog2 = (kTableN - 1) / (kLog2ZHi - kLog2ZLo);
constexpr uint32_t kTableMagic = 0x51454454u;
constexpr int kBoundOctaves = 128;  // pair-rate bound for chi in [2^(e-1), 2^e), e = -64..63
constexpr int kBoundOffset = 64;
constexpr int kBoundSub = 16;       // equal sub-intervals of each octave
constexpr int kBoundEntries = kBoundOctaves * kBoundSub;
constexpr double kNearThreshold = 1e-12;

// Layout of the tables buffer (see qed_build_tables).
struct alignas(256) DevTables {
  double2 ab64[kTableN];  // (e^z A(z), e^z B(z)) at node i
  double2 bc64[kTableN];  // (e^z B(z), e^z C(z))
  float2 ab32[kTableN];
  float2 bc32[kTableN];
  double pair_bound64[kBoundEntries];  // sup over delta of the pair-rate bracket
  float pair_bound32[kBoundEntries];
  double series[8];  // b0, b1, c0, c1, c2: small-z series of K_{2/3} and int K_{1/3}
  uint32_t magic;
  uint32_t reserved[63];
};

// ------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11).  Each round is two 32x32->64 products
// (v_mad_u64_u32 on CDNA) and XORs; the key follows a Weyl sequence.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t m0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t m1 = (uint64_t)0xCD9E8D57u * c.z;
    c = make_uint4((uint32_t)(m1 >> 32) ^ c.y ^ k0, (uint32_t)m1, (uint32_t)(m0 >> 32) ^ c.w ^ k1,
                   (uint32_t)m0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// Open-interval uniforms from the 64-bit word hi:lo.
// FP64: (m + 1/2) 2^-52 with m the top 52 bits, built from the exponent field of 1.0.
__device__ __forceinline__ double uniform64(uint32_t lo, uint32_t hi) {
  const uint64_t m = ((((uint64_t)hi) << 32) | lo) >> 12;
  const double one_plus = __longlong_as_double((long long)(0x3FF0000000000000ull | m));
  return (one_plus - 1.0) + 0x1p-53;
}
// FP32: (m + 1/2) 2^-23 with m the top 23 bits of the same word.
__device__ __forceinline__ float uniform32(uint32_t hi) {
  const float one_plus = __uint_as_float(0x3F800000u | (hi >> 9));
  return (one_plus - 1.0f) + 0x1p-24f;
}

// Counter layout shared by the event draw and the child ids:
//   key = particle id, counter = (step, sub-step | purpose << 16 | run << 24, seed lo, seed hi),
// run = the run of the reverse mode of Sec. VI (0 for the ordinary generator).  A sub-step
// code carries the run in its top byte (sub_code), so that records keep both in one word.
enum Purpose : uint32_t {
  kDraw = 0, kPhotonChild = 1, kElectronChild = 2, kPositronChild = 3, kThin = 4,
  kGenPhoton = 5, kGenPair = 6,  // generator-factor draws (Sec. VI)
  kSchwinger = 7, kSchwingerPos = 8, kSchwingerElectron = 9, kSchwingerPositron = 10,
  kThinCell = 11,   // thinning per cell block
  kPhase = 12,      // phase of the deterministic generator factor (Sec. VI)
  kThinParent = 13  // the cap on the children of one parent in one step (Sec. VII)
};

__device__ __forceinline__ uint32_t sub_code(int k, int run) {
  return (uint32_t)k | ((uint32_t)run << 24);
}

__device__ __forceinline__ uint4 draw_words(uint64_t id, uint64_t seed, uint32_t step, uint32_t sub,
                                            uint32_t purpose) {
  return philox4x32_10(make_uint4(step, (sub & 0xFF00FFFFu) | (purpose << 16), (uint32_t)seed,
                                  (uint32_t)(seed >> 32)),
                       (uint32_t)id, (uint32_t)(id >> 32));
}

__device__ __forceinline__ uint64_t child_id(uint64_t parent, uint64_t seed, uint32_t step,
                                             uint32_t sub, uint32_t purpose) {
  const uint4 o = draw_words(parent, seed, step, sub, purpose);
  uint64_t id = ((((uint64_t)o.y) << 32) | o.x) | (1ull << 63);
  return id == QED_ID_DEAD ? QED_ID_DEAD - 1 : id;
}

__device__ __forceinline__ uint32_t birth_code(uint32_t step, uint32_t sub) {
  return ((step + 1u) << 14) | (sub & 0x3FFFu);
}

// Tunable generator factor (Sec. VI): does the generator that fired for `parent` at this
// sub-step create its children?  Probability inv_fg = 1 / f_g, from the parent's own draw
// for `purpose` (kGenPhoton, kGenPair), independent of the event's (r1, r2).
__device__ __forceinline__ bool generator_runs(uint64_t parent, uint64_t seed, uint32_t step,
                                               uint32_t sub, uint32_t purpose, double inv_fg) {
  const uint4 o = draw_words(parent, seed, step, sub, purpose);
  return uniform64(o.x, o.y) < inv_fg;
}

// Deterministic form (Sec. VI, once every F occasions): the children of the parent's event
// number e are created iff (e + phi) mod F == 0, with the phase phi = (o.x F) >> 32 in
// [0, F) from the parent's own draw at step word 0, the same over its life.
__device__ __forceinline__ bool generator_every(uint64_t parent, uint64_t seed, uint32_t e,
                                                uint32_t F) {
  const uint4 o = draw_words(parent, seed, 0u, 0u, kPhase);
  const uint32_t phi = (uint32_t)(((uint64_t)o.x * (uint64_t)F) >> 32);
  return ((uint64_t)e + (uint64_t)phi) % (uint64_t)F == 0ull;
}

// ------------------------------------------------------------------------------------
// Rate brackets.  With z the argument of the synchrotron functions,
//   emission (Eq. (24)):  P = dtfac / (sqrt(3) pi gamma) * [A(z) + c B(z)],
//                         z = 2 delta / (3 chi (1 - delta)), c = delta^2 / (1 - delta)
//   pairs    (Eq. (30)):  P = dtfac / (sqrt(3) pi |k|)  * [c B(z) + C(z)],
//                         z = 2 / (3 chi d (1 - d)),      c = d/(1-d) + (1-d)/d
// (Eq. (30)'s two negative factors multiplied out; int K_{5/3} = 2 K_{2/3} - int K_{1/3}.)
// `tab` is the LDS copy of the (first, second) node pairs.
// ------------------------------------------------------------------------------------
struct Series64 {
  double b0, b1, c0, c1, c2;
};

__device__ __forceinline__ void series_bc(const Series64& s, double z, double& b, double& c) {
  const double z23 = cbrt(z * z);
  const double z43 = z23 * z23;
  b = s.b0 / z23 + s.b1 * z23 + 0.75 * s.b0 * z43;
  c = s.c0 - s.c1 * z23 - s.c2 * z43;
}

// A(z) + cB * B(z)
__device__ __forceinline__ double emission_bracket64(const double2* tab, const Series64& s,
                                                     double z, double cB) {
  if (z >= kZLo && z < kZHi) {
    const double u = (log2(z) - kLog2ZLo) * kNodesPerLog2;
    const int i = min((int)u, kTableN - 2);
    const double f = u - (double)i;
    const double2 g0 = tab[i];
    const double2 g1 = tab[i + 1];
    const double ga = g0.x + f * (g1.x - g0.x);
    const double gb = g0.y + f * (g1.y - g0.y);
    return (ga + cB * gb) * exp(-z);
  }
  if (z >= kZHi) return 0.0;
  if (z > 0.0) {
    double b, c;
    series_bc(s, z, b, c);
    return (2.0 * b - c) + cB * b;
  }
  return z == 0.0 ? __builtin_inf() : z;  // NaN propagates
}

// cB * B(z) + C(z)
__device__ __forceinline__ double pair_bracket64(const double2* tab, const Series64& s, double z,
                                                 double cB) {
  if (z >= kZLo && z < kZHi) {
    const double u = (log2(z) - kLog2ZLo) * kNodesPerLog2;
    const int i = min((int)u, kTableN - 2);
    const double f = u - (double)i;
    const double2 g0 = tab[i];
    const double2 g1 = tab[i + 1];
    const double gb = g0.x + f * (g1.x - g0.x);
    const double gc = g0.y + f * (g1.y - g0.y);
    return (cB * gb + gc) * exp(-z);
  }
  if (z >= kZHi) return 0.0;
  if (z > 0.0) {
    double b, c;
    series_bc(s, z, b, c);
    return cB * b + c;
  }
  return z == 0.0 ? __builtin_inf() : z;
}

struct Series32 {
  float b0, b1, c0, c1, c2;
};

__device__ __forceinline__ float emission_bracket32(const float2* tab, const Series32& s, float z,
                                                    float cB) {
  if (z >= (float)kZLo && z < (float)kZHi) {
    const float u = (__log2f(z) - (float)kLog2ZLo) * (float)kNodesPerLog2;
    const int i = min((int)u, kTableN - 2);
    const float f = u - (float)i;
    const float2 g0 = tab[i];
    const float2 g1 = tab[i + 1];
    const float ga = g0.x + f * (g1.x - g0.x);
    const float gb = g0.y + f * (g1.y - g0.y);
    return (ga + cB * gb) * __expf(-z);
  }
  if (z >= (float)kZHi) return 0.0f;
  if (z > 0.0f) {
    const float z23 = cbrtf(z * z);
    const float z43 = z23 * z23;
    const float b = s.b0 / z23 + s.b1 * z23 + 0.75f * s.b0 * z43;
    const float c = s.c0 - s.c1 * z23 - s.c2 * z43;
    return (2.0f * b - c) + cB * b;
  }
  return z == 0.0f ? __builtin_inff() : z;
}

__device__ __forceinline__ float pair_bracket32(const float2* tab, const Series32& s, float z,
                                                float cB) {
  if (z >= (float)kZLo && z < (float)kZHi) {
    const float u = (__log2f(z) - (float)kLog2ZLo) * (float)kNodesPerLog2;
    const int i = min((int)u, kTableN - 2);
    const float f = u - (float)i;
    const float2 g0 = tab[i];
    const float2 g1 = tab[i + 1];
    const float gb = g0.x + f * (g1.x - g0.x);
    const float gc = g0.y + f * (g1.y - g0.y);
    return (cB * gb + gc) * __expf(-z);
  }
  if (z >= (float)kZHi) return 0.0f;
  if (z > 0.0f) {
    const float z23 = cbrtf(z * z);
    const float z43 = z23 * z23;
    const float b = s.b0 / z23 + s.b1 * z23 + 0.75f * s.b0 * z43;
    const float c = s.c0 - s.c1 * z23 - s.c2 * z43;
    return cB * b + c;
  }
  return z == 0.0f ? __builtin_inff() : z;
}

// ------------------------------------------------------------------------------------
// Kinematics (FP64 in both precision modes).
// ------------------------------------------------------------------------------------
struct V3 {
  double x, y, z;
};

__device__ __forceinline__ V3 cross(const V3& a, const V3& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ double dot(const V3& a, const V3& b) {
  return a.x * b.x + a.y * b.y + a.z * b.z;
}

// chi = eps_r sqrt((gamma E + p x B)^2 - (p.E)^2), Eq. (4); for photons gamma -> |k|.
__device__ __forceinline__ double chi_of(const V3& p, double energy, const V3& E, const V3& B,
                                         double eps_r) {
  const V3 pb = cross(p, B);
  const V3 v = {energy * E.x + pb.x, energy * E.y + pb.y, energy * E.z + pb.z};
  const double pe = dot(p, E);
  const double r = dot(v, v) - pe * pe;
  return eps_r * sqrt(r > 0.0 ? r : 0.0);
}

// Boris push (Appendix A): half E kick, B rotation, half E kick; charge q = +-1.
__device__ __forceinline__ void boris(V3& p, double qh2, const V3& E, const V3& B) {
  // qh2 = q h / 2
  V3 pm = {p.x + qh2 * E.x, p.y + qh2 * E.y, p.z + qh2 * E.z};
  const double ig = qh2 / sqrt(1.0 + dot(pm, pm));
  const V3 t = {ig * B.x, ig * B.y, ig * B.z};
  const double sfac = 2.0 / (1.0 + dot(t, t));
  const V3 c1 = cross(pm, t);
  const V3 pp = {pm.x + c1.x, pm.y + c1.y, pm.z + c1.z};
  const V3 s = {sfac * t.x, sfac * t.y, sfac * t.z};
  const V3 c2 = cross(pp, s);
  p = {pm.x + c2.x + qh2 * E.x, pm.y + c2.y + qh2 * E.y, pm.z + c2.z + qh2 * E.z};
}

// dt / dt_q for leptons: dt_q = kappa 14 (2 pi eps_r) (gamma/chi)^(2/3) (Eq. (29), Eq. (6)).
__device__ __forceinline__ double substep_ratio_lepton(double dt, double chi, double gamma,
                                                       double inv_lep_scale) {
  const double r = chi / gamma;
  return dt * cbrt(r * r) * inv_lep_scale;  // inv_lep_scale = 1/(kappa 28 pi eps_r)
}
// (h / (kappa 28 pi eps_r))^3: a sub-step of length h satisfies Eq. (29) in a state of
// (chi, gamma) iff this times chi^2 is at most gamma^2 (no cube root on the sub-step path).
__device__ __forceinline__ double substep_cube(double h, double inv_lep_scale) {
  const double r = h * inv_lep_scale;
  return r * r * r;
}
// dt / dt_q for photons: dt_q = kappa 130 (2 pi eps_r) |k| / chi_g (Eq. (33)).
__device__ __forceinline__ double substep_ratio_photon(double dt, double chi_g, double kabs,
                                                       double inv_pho_scale) {
  return dt * (chi_g / kabs) * inv_pho_scale;  // inv_pho_scale = 1/(kappa 260 pi eps_r)
}

struct NsubInfo {
  int n;
  bool near_int;
  bool clamped;
};

__device__ __forceinline__ NsubInfo nsub_from_ratio(double r) {
  NsubInfo o{1, false, false};
  const double nr = rint(r);
  o.near_int = (nr >= 1.0) && fabs(r - nr) <= 1e-12 * nr;
  if (r > 1.0) {
    const double c = ceil(r);
    if (c > (double)QED_NSUB_MAX) {
      o.n = QED_NSUB_MAX;
      o.clamped = true;
    } else {
      o.n = (int)c;
    }
  }
  return o;
}

// Cell-in-cell (trilinear) interpolation on a periodic grid.  Per axis, one coordinate s
// in cell units gives the lower node i0 = floor(s) (wrapped into [0, n)), the upper node
// i1 and the fraction s - floor(s).  Each Yee component sits at node or half-node offsets
// per axis, so six such axes (node and half-node for x, y, z) serve all six components.
struct CicAxis {
  int i0, i1;
  double f;
};

__device__ __forceinline__ CicAxis cic_axis(double s, int n) {
  const double fl = floor(s);
  CicAxis a;
  a.f = s - fl;
  int i;
  if (fabs(fl) < 1073741824.0) {
    i = (int)fl;
    if ((unsigned)i >= (unsigned)n) {  // outside the primary box: wrap
      i %= n;
      if (i < 0) i += n;
    }
  } else {
    long long l = (long long)fl % n;
    if (l < 0) l += n;
    i = (int)l;
  }
  a.i0 = i;
  a.i1 = i + 1 == n ? 0 : i + 1;
  return a;
}

// The two x-neighbours g[r + i0] and g[r + i1] of one grid row (nx >= 2).  Rows are
// contiguous in x, so the pair comes from one 8-byte buffer load (4-byte aligned, which
// buffer loads allow): 4 loads per component instead of 8 in the scattered gathers that
// bound the grid kernels.  Where the pair wraps round the periodic boundary (i0 = nx - 1,
// i1 = 0) the load covers (nx - 2, nx - 1) instead, and g[r] is read on its own.  The
// buffer descriptor spans the grid, so byte offsets are 32-bit: grids of 2^30 values or
// more take the plain path below.  (A plain 8-byte load at 4-byte alignment is split into
// two by the compiler; the buffer load is not.)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t cic_rsrc(const float* g, unsigned values) {
  // word 3 0x00020000: raw 32-bit data format on gfx9-family targets.  The size (bytes)
  // and the offsets below are unsigned 32-bit in the descriptor; the int casts keep the bits.
  return __builtin_amdgcn_make_buffer_rsrc((void*)g, 0, (int)(values * 4u), 0x00020000);
}

__device__ __forceinline__ float2 cic_pair(__amdgpu_buffer_rsrc_t rs, const float* __restrict__ g,
                                           int r, const CicAxis& ax) {
  const bool wrap = ax.i1 == 0;
  const unsigned b = (unsigned)(r + ax.i0 - (wrap ? 1 : 0));
  const float2 p = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)(b * 4u), 0, 0));
  float2 v = make_float2(wrap ? p.y : p.x, p.y);
  if (wrap) v.y = g[r];
  return v;
}

// One component: 8 grid values around the point, interpolated along x, then y, then z.
// nxy = nx * ny; the grid holds fewer than 2^31 values (nall of them).  PAIRED takes the
// x-neighbours in pairs (the photon kernels, which the gathers bound); the lepton kernel
// gathers once per step between sub-steps that dominate its time, and the pairs' extra
// registers in flight cost it more than they save.
template <bool PAIRED>
__device__ __forceinline__ double cic_component(const float* __restrict__ g, const CicAxis& ax,
                                                const CicAxis& ay, const CicAxis& az, int nx,
                                                int nxy, int nall) {
  const int z0 = az.i0 * nxy, z1 = az.i1 * nxy;
  const int y0 = ay.i0 * nx, y1 = ay.i1 * nx;
  const int r00 = z0 + y0, r01 = z0 + y1, r10 = z1 + y0, r11 = z1 + y1;
  double v000, v100, v010, v110, v001, v101, v011, v111;
  if (PAIRED && nall < (1 << 30)) {
    const __amdgpu_buffer_rsrc_t rs = cic_rsrc(g, (unsigned)nall);
    const float2 p00 = cic_pair(rs, g, r00, ax), p01 = cic_pair(rs, g, r01, ax);
    const float2 p10 = cic_pair(rs, g, r10, ax), p11 = cic_pair(rs, g, r11, ax);
    v000 = p00.x, v100 = p00.y, v010 = p01.x, v110 = p01.y;
    v001 = p10.x, v101 = p10.y, v011 = p11.x, v111 = p11.y;
  } else {
    v000 = g[r00 + ax.i0], v100 = g[r00 + ax.i1], v010 = g[r01 + ax.i0], v110 = g[r01 + ax.i1];
    v001 = g[r10 + ax.i0], v101 = g[r10 + ax.i1], v011 = g[r11 + ax.i0], v111 = g[r11 + ax.i1];
  }
  const double fx = ax.f, fy = ay.f, fz = az.f;
  const double c00 = v000 + fx * (v100 - v000);
  const double c10 = v010 + fx * (v110 - v010);
  const double c01 = v001 + fx * (v101 - v001);
  const double c11 = v011 + fx * (v111 - v011);
  const double c0 = c00 + fy * (c10 - c00);
  const double c1 = c01 + fy * (c11 - c01);
  return c0 + fz * (c1 - c0);
}

struct FieldArgs {
  int kind;
  double amp, omega, phase, tn;
  const float* grid[6];
  int n[3];
  double inv_dx[3], origin[3];
};

// Fields at position x for the kinds that depend on position (CP standing wave, Yee).
// Space-independent kinds are evaluated once per instance by the step's prep kernel.
template <bool PAIRED = false>
__device__ __forceinline__ void field_at_position(const FieldArgs& f, double inst_amp, const V3& x,
                                                  V3& E, V3& B) {
  if (f.kind == QED_FIELD_LP_STANDING) {
    const double a1 = f.amp * inst_amp;
    double sph, cph, skx, ckx;
    sincos(f.omega * f.tn + f.phase, &sph, &cph);
    sincos(f.omega * x.x, &skx, &ckx);
    E = {0.0, a1 * skx * cph, 0.0};
    B = {0.0, 0.0, -a1 * ckx * sph};
    return;
  }
  if (f.kind == QED_FIELD_CP_STANDING) {
    const double a2 = 2.0 * f.amp * inst_amp;
    double sph, cph, skx, ckx;
    sincos(f.omega * f.tn + f.phase, &sph, &cph);
    sincos(f.omega * x.x, &skx, &ckx);
    E = {0.0, a2 * ckx * cph, a2 * ckx * sph};
    B = {0.0, a2 * skx * cph, a2 * skx * sph};
    return;
  }
  // QED_FIELD_YEE: Ex at (i+1/2, j, k), Ey (i, j+1/2, k), Ez (i, j, k+1/2),
  // Bx (i, j+1/2, k+1/2), By (i+1/2, j, k+1/2), Bz (i+1/2, j+1/2, k)
  const double sx = (x.x - f.origin[0]) * f.inv_dx[0];
  const double sy = (x.y - f.origin[1]) * f.inv_dx[1];
  const double sz = (x.z - f.origin[2]) * f.inv_dx[2];
  const int nx = f.n[0], ny = f.n[1], nz = f.n[2], nxy = nx * ny, nall = nxy * nz;
  const CicAxis x0 = cic_axis(sx, nx), xh = cic_axis(sx - 0.5, nx);
  const CicAxis y0 = cic_axis(sy, ny), yh = cic_axis(sy - 0.5, ny);
  const CicAxis z0 = cic_axis(sz, nz), zh = cic_axis(sz - 0.5, nz);
  E.x = cic_component<PAIRED>(f.grid[0], xh, y0, z0, nx, nxy, nall);
  E.y = cic_component<PAIRED>(f.grid[1], x0, yh, z0, nx, nxy, nall);
  E.z = cic_component<PAIRED>(f.grid[2], x0, y0, zh, nx, nxy, nall);
  B.x = cic_component<PAIRED>(f.grid[3], x0, yh, zh, nx, nxy, nall);
  B.y = cic_component<PAIRED>(f.grid[4], xh, y0, zh, nx, nxy, nall);
  B.z = cic_component<PAIRED>(f.grid[5], xh, yh, z0, nx, nxy, nall);
}

// ------------------------------------------------------------------------------------
// Wavefront helpers (64 lanes).
// ------------------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }
__device__ __forceinline__ uint64_t lanes_below() {
  return (1ull << lane_id()) - 1ull;
}
__device__ __forceinline__ uint64_t wave_ballot(bool b) { return __ballot(b); }

template <typename T>
__device__ __forceinline__ T wave_bcast(T v, int src) {
  return __shfl(v, src, 64);
}

__device__ __forceinline__ void atomic_max_nonneg(double* addr, double v) {
  // non-negative doubles order like their bit patterns
  if (v > 0.0) atomicMax((unsigned long long*)addr, (unsigned long long)__double_as_longlong(v));
}

}  // namespace qedk
