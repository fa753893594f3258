// Device-side building blocks of the MI355X quark-solve library: complex
// arithmetic, the even/odd structure-of-arrays field layouts in FP64, FP32 and
// FP16 (with a per-site norm), the spin projectors of the Wilson hopping term,
// and the FP64 wavefront/workgroup reductions.
//
// Layouts (all "site fastest", so that the 64 lanes of a wavefront touch 64
// consecutive sites of one right-hand side and every load is coalesced):
//
//   spinor chunk array  [rhs][parity][chunk][site]    (16-byte chunks)
//       FP64: 12 chunks of one complex (double2)
//       FP32:  6 chunks of two complex (float4)
//       FP16:  3 chunks of four complex (8 x fp16), plus a norm array
//              [rhs][parity][site] (fp32): stored value = value / norm,
//              norm = max |real component| of the 24 reals of the site.
//   link array          FP64 [parity][mu][9][site] (double2); FP32 / FP16
//                       [parity][mu][3][site] chunks of the first two rows
//
// The [site] dimension of every array has the padded length Geom::vs >= vh
// (the padding is never read or written).
//
// A "site" is a half-lattice index s = xh + (Lx/2)(y + Ly(z + Lz t)) over the
// dynamical time slices t = 0..Td-1 (x0 = t + 1 under Schroedinger-functional
// boundaries, x0 = t otherwise); its x coordinate is 2 xh + ((x0+y+z+p) & 1).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mfq {

typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------- complex
template <typename T>
struct cpx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cpx<T> operator-(cpx<T> a) { return {-a.re, -a.im}; }
template <typename T>
__device__ __forceinline__ cpx<T> operator*(T s, cpx<T> a) { return {s * a.re, s * a.im}; }
// a * b
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
template <typename T>
__device__ __forceinline__ cpx<T> cjmul(cpx<T> a, cpx<T> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// i * a
template <typename T>
__device__ __forceinline__ cpx<T> imul(cpx<T> a) { return {-a.im, a.re}; }
template <typename T>
__device__ __forceinline__ T norm2(cpx<T> a) { return a.re * a.re + a.im * a.im; }

// ---------------------------------------------------------------- geometry
enum : int { BC_SF = 0, BC_PERIODIC = 1, BC_ANTIPERIODIC = 2 };

struct Geom {
  int lx, ly, lz, td;  // spatial extents and number of dynamical time slices
  int lxh;             // lx / 2
  int vh;              // half volume of the dynamical lattice
  int t0;              // x0 of the first dynamical slice (1 for SF, else 0)
  int bc;
  // Storage stride (in sites) of every SoA component array: vh rounded up to
  // 16 times an odd number, so the arrays of one site start an odd number of
  // 256-byte granules apart.  With a power-of-two stride (vh = 2^20 at
  // 32^3 x 64) all components of a site fall in one L2 channel and set and
  // evict each other.
  int vs;
  // Parities the vector kernels cover: 2 (every site), or 1 (the even sites
  // only: the even/odd Schur-complement solves).
  int npar;
  // Division by lxh, ly, lz without a divide: q = umulhi(2n, m) with
  // m = ceil(2^31 / d) equals n / d whenever n * d < 2^31 (set by geom_init).
  unsigned mxh, my, mz;
  // Half-index strides of y, z and t, and the jumps of a periodic wrap.
  int sy, sz, st;
  int wy, wz, wt;  // (ly - 1) sy, (lz - 1) sz, (td - 1) st
};

// n / d for the divisors of Geom (n * d < 2^31), and the remainder.
__device__ __forceinline__ int fdiv(int n, unsigned m) { return (int)__umulhi(2u * (unsigned)n, m); }

inline unsigned fdiv_magic(int d) { return (unsigned)(((1ull << 31) + (unsigned)d - 1) / (unsigned)d); }

// Fills the derived fields of g from lx, ly, lz, td.
inline void geom_init(Geom& g) {
  g.lxh = g.lx / 2;
  g.vh = g.lxh * g.ly * g.lz * g.td;
  g.mxh = fdiv_magic(g.lxh);
  g.my = fdiv_magic(g.ly);
  g.mz = fdiv_magic(g.lz);
  g.sy = g.lxh;
  g.sz = g.lxh * g.ly;
  g.st = g.sz * g.lz;
  g.wy = (g.ly - 1) * g.sy;
  g.wz = (g.lz - 1) * g.sz;
  g.wt = (g.td - 1) * g.st;
}

struct Coords {
  int x, y, z, t;
};

__device__ __forceinline__ Coords site_coords(const Geom& g, int s, int parity) {
  Coords c;
  int r = fdiv(s, g.mxh);
  const int xh = s - r * g.lxh;
  int q = fdiv(r, g.my);
  c.y = r - q * g.ly;
  c.t = fdiv(q, g.mz);
  c.z = q - c.t * g.lz;
  c.x = 2 * xh + ((c.t + g.t0 + c.y + c.z + parity) & 1);
  return c;
}

__device__ __forceinline__ int half_index(const Geom& g, int x, int y, int z, int t) {
  return (x >> 1) + g.lxh * (y + g.ly * (z + g.lz * t));
}

// ------------------------------------------------------------- storage traits
template <typename S>
struct Store;

template <>
struct Store<double> {
  using chunk = d2;
  static constexpr int NC = 12;
  using link_elem = d2;
};
template <>
struct Store<float> {
  using chunk = f4;
  static constexpr int NC = 6;
  using link_elem = f2;
};
template <>
struct Store<_Float16> {
  using chunk = h8;
  static constexpr int NC = 3;
  using link_elem = h2;
};

// A batched spinor field: n_rhs full (both parity) fields.
template <typename S>
struct Field {
  typename Store<S>::chunk* data;
  float* norm;  // FP16 only
  int vh;
  __device__ __forceinline__ long cidx(int rhs, int par, int c, int s) const {
    return ((long)(rhs * 2 + par) * Store<S>::NC + c) * vh + s;
  }
  __device__ __forceinline__ long nidx(int rhs, int par, int s) const {
    return (long)(rhs * 2 + par) * vh + s;
  }
  // Start of component array c of (rhs, par).  When rhs and par are uniform
  // over the wavefront this is a scalar address, and an element is reached
  // with a 32-bit per-lane byte offset (see at()).
  __device__ __forceinline__ typename Store<S>::chunk* comp(int rhs, int par, int c) const {
    return data + (long)((rhs * 2 + par) * Store<S>::NC + c) * vh;
  }
};

// Element s of an array that starts at base: scalar base + 32-bit lane offset
// (s < 2^27, so the byte offset fits in 32 bits).
template <typename C>
__device__ __forceinline__ C& at(C* base, int s) {
  return *(C*)((char*)base + (unsigned)s * (unsigned)sizeof(C));
}
template <typename C>
__device__ __forceinline__ const C& at(const C* base, int s) {
  return *(const C*)((const char*)base + (unsigned)s * (unsigned)sizeof(C));
}

// Links of one precision.  FP64: full layout [parity][mu][9][site], one
// complex per element.  FP32 and FP16 (the inner-solver copies, SU(3) links
// only): the first two rows, [parity][mu][3][site] of 16-byte (FP32) or
// 8-byte (FP16) chunks of two complex numbers; the third row is rebuilt as the
// complex conjugate of the cross product of the first two, so a link costs
// 48 (FP32) or 24 (FP16) bytes and three loads.
template <typename S>
struct Links {
  const typename Store<S>::link_elem* data;  // [parity][mu][9][vh] (full layout)
  int vh;
  int comp;  // 1 for the two-row layout (FP32 / FP16)
  __device__ __forceinline__ long idx(int par, int mu, int k, int s) const {
    return ((long)(par * 4 + mu) * 9 + k) * vh + s;
  }
  __device__ __forceinline__ long cidx(int par, int mu, int c, int s) const {
    return ((long)(par * 4 + mu) * 3 + c) * vh + s;
  }
  __device__ __forceinline__ const typename Store<S>::link_elem* row(int par, int mu, int k) const {
    return data + (long)((par * 4 + mu) * 9 + k) * vh;
  }
};


// Spinor register block: v[3 * spin + colour].
template <typename T>
struct Spinor {
  cpx<T> v[12];
};

template <typename T>
__device__ __forceinline__ void load_spinor(const Field<double>& f, int rhs, int par, int s, Spinor<T>& o) {
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    d2 q = at(f.comp(rhs, par, c), s);
    o.v[c] = {(T)q.x, (T)q.y};
  }
}
template <typename T>
__device__ __forceinline__ void load_spinor(const Field<float>& f, int rhs, int par, int s, Spinor<T>& o) {
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    f4 q = at(f.comp(rhs, par, c), s);
    o.v[2 * c] = {(T)q.x, (T)q.y};
    o.v[2 * c + 1] = {(T)q.z, (T)q.w};
  }
}
// FP16 storage without its per-site norm: the caller applies the norm.
template <typename T>
__device__ __forceinline__ void load_spinor_raw(const Field<_Float16>& f, int rhs, int par, int s, Spinor<T>& o) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    h8 q = at(f.comp(rhs, par, c), s);
#pragma unroll
    for (int k = 0; k < 4; ++k) o.v[4 * c + k] = {(T)(float)q[2 * k], (T)(float)q[2 * k + 1]};
  }
}
__device__ __forceinline__ float load_norm(const Field<_Float16>& f, int rhs, int par, int s) {
  return at(f.norm + (long)(rhs * 2 + par) * f.vh, s);
}
template <typename T>
__device__ __forceinline__ void load_spinor(const Field<_Float16>& f, int rhs, int par, int s, Spinor<T>& o) {
  const float n = load_norm(f, rhs, par, s);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    h8 q = at(f.comp(rhs, par, c), s);
#pragma unroll
    for (int k = 0; k < 4; ++k) o.v[4 * c + k] = {(T)((float)q[2 * k] * n), (T)((float)q[2 * k + 1] * n)};
  }
}

template <typename T>
__device__ __forceinline__ void store_spinor(const Field<double>& f, int rhs, int par, int s, const Spinor<T>& o) {
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    d2 q;
    q.x = (double)o.v[c].re;
    q.y = (double)o.v[c].im;
    at(f.comp(rhs, par, c), s) = q;
  }
}
template <typename T>
__device__ __forceinline__ void store_spinor(const Field<float>& f, int rhs, int par, int s, const Spinor<T>& o) {
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    f4 q;
    q.x = (float)o.v[2 * c].re;
    q.y = (float)o.v[2 * c].im;
    q.z = (float)o.v[2 * c + 1].re;
    q.w = (float)o.v[2 * c + 1].im;
    at(f.comp(rhs, par, c), s) = q;
  }
}
template <typename T>
__device__ __forceinline__ void store_spinor(const Field<_Float16>& f, int rhs, int par, int s, const Spinor<T>& o) {
  float m = 0.f;
#pragma unroll
  for (int c = 0; c < 12; ++c) m = fmaxf(m, fmaxf(fabsf((float)o.v[c].re), fabsf((float)o.v[c].im)));
  const float inv = m > 0.f ? 1.0f / m : 0.f;
  at(f.norm + (long)(rhs * 2 + par) * f.vh, s) = m;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    h8 q;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      q[2 * k] = (_Float16)((float)o.v[4 * c + k].re * inv);
      q[2 * k + 1] = (_Float16)((float)o.v[4 * c + k].im * inv);
    }
    at(f.comp(rhs, par, c), s) = q;
  }
}

// ------------------------------------------------ buffer loads (scalar base)
// A raw buffer resource over `bytes` bytes from base (no stride; the last
// word is the gfx9-family default for untyped loads).  It lives in scalar
// registers, so base must be uniform over the wavefront; every load names a
// 32-bit lane offset and a 32-bit scalar offset, and a load past `bytes`
// returns zero instead of touching memory.
using rsrc_t = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ rsrc_t buf_rsrc(const void* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
template <typename C>
__device__ __forceinline__ C buf_load(rsrc_t r, unsigned voff, unsigned soff) {
  if constexpr (sizeof(C) == 16)
    return __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
  else if constexpr (sizeof(C) == 8)
    return __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  else
    return __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

// The spinor at site s of (rhs, par) through one buffer resource for the
// whole (rhs, par) field: the components share the lane offset and differ by
// a scalar one.  rhs and par must be uniform over the wavefront, and the
// field of one (rhs, par) must span less than 4 GiB (the lattice limit).
template <typename T>
__device__ __forceinline__ void buf_load_spinor(const Field<double>& f, int rhs, int par, int s, Spinor<T>& o) {
  const unsigned cb = (unsigned)f.vh * 16u;
  const rsrc_t rs = buf_rsrc(f.comp(rhs, par, 0), 12u * cb);
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const d2 q = buf_load<d2>(rs, (unsigned)s * 16u, c * cb);
    o.v[c] = {(T)q.x, (T)q.y};
  }
}
template <typename T>
__device__ __forceinline__ void buf_load_spinor(const Field<float>& f, int rhs, int par, int s, Spinor<T>& o) {
  const unsigned cb = (unsigned)f.vh * 16u;
  const rsrc_t rs = buf_rsrc(f.comp(rhs, par, 0), 6u * cb);
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const f4 q = buf_load<f4>(rs, (unsigned)s * 16u, c * cb);
    o.v[2 * c] = {(T)q.x, (T)q.y};
    o.v[2 * c + 1] = {(T)q.z, (T)q.w};
  }
}
// FP16: the raw components; the site's norm is returned for the caller to apply.
template <typename T>
__device__ __forceinline__ float buf_load_spinor_raw(const Field<_Float16>& f, int rhs, int par, int s, Spinor<T>& o) {
  const unsigned cb = (unsigned)f.vh * 16u;
  const rsrc_t rs = buf_rsrc(f.comp(rhs, par, 0), 3u * cb);
  const rsrc_t rn = buf_rsrc(f.norm + (long)(rhs * 2 + par) * f.vh, (unsigned)f.vh * 4u);
  const float n = buf_load<float>(rn, (unsigned)s * 4u, 0);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const h8 q = buf_load<h8>(rs, (unsigned)s * 16u, c * cb);
#pragma unroll
    for (int k = 0; k < 4; ++k) o.v[4 * c + k] = {(T)(float)q[2 * k], (T)(float)q[2 * k + 1]};
  }
  return n;
}

// The third row of an SU(3) matrix from the first two: conj(row0 x row1),
// each component a chain of four fused multiply-adds per real part.
template <typename T>
__device__ __forceinline__ void third_row(cpx<T> u[9]) {
#define MFQ_CROSS(o, a, b, c, d) /* o = conj(a d - b c) */                                  \
  {                                                                                        \
    T re = u[a].re * u[d].re;                                                              \
    re = fma(-u[a].im, u[d].im, re);                                                       \
    re = fma(-u[b].re, u[c].re, re);                                                       \
    re = fma(u[b].im, u[c].im, re);                                                        \
    T im = -u[a].re * u[d].im;                                                             \
    im = fma(-u[a].im, u[d].re, im);                                                       \
    im = fma(u[b].re, u[c].im, im);                                                        \
    im = fma(u[b].im, u[c].re, im);                                                        \
    u[o] = {re, im};                                                                       \
  }
  MFQ_CROSS(6, 1, 2, 4, 5)
  MFQ_CROSS(7, 2, 0, 5, 3)
  MFQ_CROSS(8, 0, 1, 3, 4)
#undef MFQ_CROSS
}

template <typename T>
__device__ __forceinline__ void load_link(const Links<double>& l, int par, int mu, int s, cpx<T> u[9]) {
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    d2 q = at(l.row(par, mu, k), s);
    u[k] = {(T)q.x, (T)q.y};
  }
}
template <typename T>
__device__ __forceinline__ void load_link(const Links<float>& l, int par, int mu, int s, cpx<T> u[9]) {
  const f4* c = (const f4*)l.data;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    f4 q = at(c + (long)((par * 4 + mu) * 3 + k) * l.vh, s);
    u[2 * k] = {(T)q.x, (T)q.y};
    u[2 * k + 1] = {(T)q.z, (T)q.w};
  }
  third_row(u);
}
template <typename T>
__device__ __forceinline__ void load_link(const Links<_Float16>& l, int par, int mu, int s, cpx<T> u[9]) {
  const h4* c = (const h4*)l.data;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    h4 q = at(c + (long)((par * 4 + mu) * 3 + k) * l.vh, s);
    u[2 * k] = {(T)(float)q.x, (T)(float)q.y};
    u[2 * k + 1] = {(T)(float)q.z, (T)(float)q.w};
  }
  third_row(u);
}

// Link U_mu(s) of parity par through one buffer resource per (par, mu)
// (par uniform over the wavefront).
template <typename T>
__device__ __forceinline__ void buf_load_link(const Links<double>& l, int par, int mu, int s, cpx<T> u[9]) {
  const unsigned cb = (unsigned)l.vh * 16u;
  const rsrc_t rs = buf_rsrc(l.row(par, mu, 0), 9u * cb);
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const d2 q = buf_load<d2>(rs, (unsigned)s * 16u, k * cb);
    u[k] = {(T)q.x, (T)q.y};
  }
}
template <typename T>
__device__ __forceinline__ void buf_load_link(const Links<float>& l, int par, int mu, int s, cpx<T> u[9]) {
  const unsigned cb = (unsigned)l.vh * 16u;
  const rsrc_t rs = buf_rsrc((const f4*)l.data + (long)((par * 4 + mu) * 3) * l.vh, 3u * cb);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const f4 q = buf_load<f4>(rs, (unsigned)s * 16u, k * cb);
    u[2 * k] = {(T)q.x, (T)q.y};
    u[2 * k + 1] = {(T)q.z, (T)q.w};
  }
  third_row(u);
}
template <typename T>
__device__ __forceinline__ void buf_load_link(const Links<_Float16>& l, int par, int mu, int s, cpx<T> u[9]) {
  const unsigned cb = (unsigned)l.vh * 8u;
  const rsrc_t rs = buf_rsrc((const h4*)l.data + (long)((par * 4 + mu) * 3) * l.vh, 3u * cb);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const h4 q = buf_load<h4>(rs, (unsigned)s * 8u, k * cb);
    u[2 * k] = {(T)(float)q.x, (T)(float)q.y};
    u[2 * k + 1] = {(T)(float)q.z, (T)(float)q.w};
  }
  third_row(u);
}

// -------------------------------------------------- Wilson hopping algebra
// Chiral basis: g_mu = [[0, e_mu], [e_mu^+, 0]], e_0 = -1, e_k = -i sigma_k.
// (1 + sg g_mu) psi = [h ; sg e_mu^+ h] with h = psi_up + sg e_mu psi_down, so
// only the 2-spin "half spinor" h travels through the colour multiply.

// h = psi_up + sg * e_mu psi_down   (colour index a)
template <int MU, typename T>
__device__ __forceinline__ void project(const Spinor<T>& p, T sg, int a, cpx<T>& h0, cpx<T>& h1) {
  const cpx<T> u0 = p.v[a], u1 = p.v[3 + a], d0 = p.v[6 + a], d1 = p.v[9 + a];
  if constexpr (MU == 0) {  // e d = (-d0, -d1)
    h0 = u0 - sg * d0;
    h1 = u1 - sg * d1;
  } else if constexpr (MU == 1) {  // e d = (-i d1, -i d0)
    h0 = u0 - sg * imul(d1);
    h1 = u1 - sg * imul(d0);
  } else if constexpr (MU == 2) {  // e d = (-d1, d0)
    h0 = u0 - sg * d1;
    h1 = u1 + sg * d0;
  } else {  // e d = (-i d0, i d1)
    h0 = u0 - sg * imul(d0);
    h1 = u1 + sg * imul(d1);
  }
}

// The lower two spins of acc += [g ; sg e_mu^+ g]   (colour index a)
template <int MU, typename T>
__device__ __forceinline__ void reconstruct_lower(Spinor<T>& acc, T sg, int a, cpx<T> g0, cpx<T> g1) {
  if constexpr (MU == 0) {  // e^+ g = (-g0, -g1)
    acc.v[6 + a] = acc.v[6 + a] - sg * g0;
    acc.v[9 + a] = acc.v[9 + a] - sg * g1;
  } else if constexpr (MU == 1) {  // e^+ g = (i g1, i g0)
    acc.v[6 + a] = acc.v[6 + a] + sg * imul(g1);
    acc.v[9 + a] = acc.v[9 + a] + sg * imul(g0);
  } else if constexpr (MU == 2) {  // e^+ g = (g1, -g0)
    acc.v[6 + a] = acc.v[6 + a] + sg * g1;
    acc.v[9 + a] = acc.v[9 + a] - sg * g0;
  } else {  // e^+ g = (i g0, -i g1)
    acc.v[6 + a] = acc.v[6 + a] + sg * imul(g0);
    acc.v[9 + a] = acc.v[9 + a] - sg * imul(g1);
  }
}

// acc += [g ; sg e_mu^+ g]   (colour index a)
template <int MU, typename T>
__device__ __forceinline__ void reconstruct(Spinor<T>& acc, T sg, int a, cpx<T> g0, cpx<T> g1) {
  acc.v[a] = acc.v[a] + g0;
  acc.v[3 + a] = acc.v[3 + a] + g1;
  reconstruct_lower<MU>(acc, sg, a, g0, g1);
}

// ---------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace mfq
