// dl_common.hpp -- device-side building blocks shared by the HIP kernels:
// complex arithmetic, storage formats of spinor and link fields, even-odd
// site geometry, wavefront reductions and the XCD-aware block order.
//
// Device layouts (private to the library):
//   half-spinor field of one parity, one right-hand side: 12 complex
//   components (spin-major, then colour) in the stored spin basis (see
//   to_internal below), structure-of-arrays in 16-byte vectors of VEC
//   components (VEC = 1 for FP64, 2 for FP32, 4 for FP16 / BF16): vector j of
//   checkerboard site cb at vector index j * Vh + cb, holding the components
//   comp_of<VEC>(j, 0 .. VEC-1), so one lane's 16-byte load brings VEC
//   components and a wavefront's load covers 64 consecutive sites; nrhs
//   fields follow each other with stride rhs_stride_bytes (12 * Vh elements
//   and a gap, see there).  FP16 fields carry
//   an extra FP32 scale per site ([rhs * Vh + cb]) and store entries divided
//   by it.
//   links: [mu][parity][NE][Vh] complex with NE = 6 (rows 0-1, the third row
//   is rebuilt as the conjugated cross product) or 9.  U_mu(x) of a site x of
//   parity p sits at [mu][p][.][cb(x)].
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dl {

// ---------------------------------------------------------------- complex

template <typename R>
struct cx {
    R re, im;
};

template <typename R>
__device__ __forceinline__ cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <typename R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a) { return {-a.re, -a.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
template <typename R>
__device__ __forceinline__ cx<R> conj(cx<R> a) { return {a.re, -a.im}; }
// i * a
template <typename R>
__device__ __forceinline__ cx<R> times_i(cx<R> a) { return {-a.im, a.re}; }
// acc += a * b
template <typename R>
__device__ __forceinline__ void cmac(cx<R> &acc, cx<R> a, cx<R> b)
{
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(a.im, b.re, acc.im);
}
// acc += conj(a) * b
template <typename R>
__device__ __forceinline__ void cmac_conj(cx<R> &acc, cx<R> a, cx<R> b)
{
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(-a.im, b.re, acc.im);
}

// ---------------------------------------------------------------- storage formats

// Storage type S -> arithmetic type R and the packed complex element.
template <typename S>
struct Fmt;
template <>
struct Fmt<double> {
    using R = double;
    using E = double2;
    static constexpr bool scaled = false;
    static constexpr int VEC = 1;
    __device__ static __forceinline__ cx<double> ld(const E *p, int64_t i)
    {
        E v = p[i];
        return {v.x, v.y};
    }
    __device__ static __forceinline__ void st(E *p, int64_t i, cx<double> v) { p[i] = make_double2(v.re, v.im); }
    // the components of one 16-byte vector read as raw words
    __device__ static __forceinline__ void unpack(const uint4 &q, cx<double> v[1])
    {
        double2 d;
        __builtin_memcpy(&d, &q, 16);
        v[0] = {d.x, d.y};
    }
    __device__ static __forceinline__ uint4 pack(const cx<double> v[1])
    {
        const double2 d = make_double2(v[0].re, v[0].im);
        uint4 q;
        __builtin_memcpy(&q, &d, 16);
        return q;
    }
};
template <>
struct Fmt<float> {
    using R = float;
    using E = float2;
    static constexpr bool scaled = false;
    static constexpr int VEC = 2;
    __device__ static __forceinline__ cx<float> ld(const E *p, int64_t i)
    {
        E v = p[i];
        return {v.x, v.y};
    }
    __device__ static __forceinline__ void st(E *p, int64_t i, cx<float> v) { p[i] = make_float2(v.re, v.im); }
    __device__ static __forceinline__ void unpack(const uint4 &q, cx<float> v[2])
    {
        float4 f;
        __builtin_memcpy(&f, &q, 16);
        v[0] = {f.x, f.y};
        v[1] = {f.z, f.w};
    }
    __device__ static __forceinline__ uint4 pack(const cx<float> v[2])
    {
        const float4 f = make_float4(v[0].re, v[0].im, v[1].re, v[1].im);
        uint4 q;
        __builtin_memcpy(&q, &f, 16);
        return q;
    }
};

// four 16-bit complex numbers in one 16-byte vector, as raw 32-bit words
template <typename H2, typename CVT>
__device__ __forceinline__ void unpack16(const uint4 &q, cx<float> v[4], CVT cvt)
{
    const unsigned w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        H2 h;
        __builtin_memcpy(&h, &w[i], 4);
        const float2 f = cvt(h);
        v[i] = {f.x, f.y};
    }
}
template <typename H2, typename CVT>
__device__ __forceinline__ uint4 pack16(const cx<float> v[4], CVT cvt)
{
    unsigned w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const H2 h = cvt(make_float2(v[i].re, v[i].im));
        __builtin_memcpy(&w[i], &h, 4);
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
}
// two 16-bit complex numbers in 8 bytes
template <typename H2, typename CVT>
__device__ __forceinline__ void unpack16x2(const uint2 &q, cx<float> v[2], CVT cvt)
{
    const unsigned w[2] = {q.x, q.y};
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        H2 h;
        __builtin_memcpy(&h, &w[i], 4);
        const float2 f = cvt(h);
        v[i] = {f.x, f.y};
    }
}
template <>
struct Fmt<__half> {
    using R = float;
    using E = __half2;
    static constexpr bool scaled = true;
    __device__ static __forceinline__ cx<float> ld(const E *p, int64_t i)
    {
        float2 v = __half22float2(p[i]);
        return {v.x, v.y};
    }
    __device__ static __forceinline__ void st(E *p, int64_t i, cx<float> v)
    {
        p[i] = __float22half2_rn(make_float2(v.re, v.im));
    }
    static constexpr int VEC = 4;
    __device__ static __forceinline__ void unpack(const uint4 &q, cx<float> v[4])
    {
        unpack16<E>(q, v, [](E h) { return __half22float2(h); });
    }
    __device__ static __forceinline__ void unpack2(const uint2 &q, cx<float> v[2])
    {
        unpack16x2<E>(q, v, [](E h) { return __half22float2(h); });
    }
    __device__ static __forceinline__ uint4 pack(const cx<float> v[4])
    {
        return pack16<E>(v, [](float2 f) { return __float22half2_rn(f); });
    }
};
template <>
struct Fmt<__hip_bfloat16> {
    using R = float;
    using E = __hip_bfloat162;
    static constexpr bool scaled = false;
    __device__ static __forceinline__ cx<float> ld(const E *p, int64_t i)
    {
        float2 v = __bfloat1622float2(p[i]);
        return {v.x, v.y};
    }
    __device__ static __forceinline__ void st(E *p, int64_t i, cx<float> v)
    {
        p[i] = __float22bfloat162_rn(make_float2(v.re, v.im));
    }
    static constexpr int VEC = 4;
    __device__ static __forceinline__ void unpack(const uint4 &q, cx<float> v[4])
    {
        unpack16<E>(q, v, [](E h) { return __bfloat1622float2(h); });
    }
    __device__ static __forceinline__ void unpack2(const uint2 &q, cx<float> v[2])
    {
        unpack16x2<E>(q, v, [](E h) { return __bfloat1622float2(h); });
    }
    __device__ static __forceinline__ uint4 pack(const cx<float> v[4])
    {
        return pack16<E>(v, [](float2 f) { return __float22bfloat162_rn(f); });
    }
};

// A set of nrhs half-spinor fields of one parity.
struct Field {
    void *d;       // [nrhs][12/VEC][Vh] 16-byte vectors of the storage type
    float *nrm;    // [nrhs][Vh] per-site scale (FP16 only, else null)
};

// Spin basis of the stored fields.  Every spinor field is stored in the basis
// psi' = T psi, T = [[1, 1], [1, -1]] acting on the (upper, lower) spin pairs
// of the chiral basis.  T / sqrt 2 is real, symmetric and its own inverse,
// and the scale cancels in the operator: in this basis gamma_4 = diag(1, 1,
// -1, -1), so a temporal projector (1 +- gamma_4) keeps one spin pair and a
// temporal hop reads half of its neighbour's spinor, and gamma_k = [[0,
// i sigma_k], [-i sigma_k, 0]] (the chiral A_k = -i sigma_k with its sign
// flipped).  Inner products and norms scale by 2, so relative residuals and
// the Krylov coefficients are unchanged.  Fields cross to and from the
// canonical basis through to_internal / to_canonical; the factor 1/2 is
// exact, so a complex Z2 or unit source survives the round trip bit for bit.
template <typename R>
__device__ __forceinline__ void to_internal(cx<R> v[12])
{
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const cx<R> u = v[k], d = v[6 + k];
        v[k] = u + d;
        v[6 + k] = u - d;
    }
}
template <typename R>
__device__ __forceinline__ void to_canonical(cx<R> v[12])
{
    const R h = R(0.5);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const cx<R> u = v[k], d = v[6 + k];
        v[k] = h * (u + d);
        v[6 + k] = h * (u - d);
    }
}

// The component (3 spin + colour) held by entry q of 16-byte vector j of a
// stored spinor with VEC entries per vector.  VEC = 1 and 2 keep the
// components in order.  The 16-bit formats (VEC = 4) hold {0, 1, 2, 3},
// {6, 7, 8, 9} and {4, 5, 10, 11}: the upper spin pair (0-5) is then vector 0
// and the low 8 bytes of vector 2, the lower pair (6-11) vector 1 and the high
// 8 bytes of vector 2, so either pair loads as 24 contiguous-per-lane bytes.
template <int V>
__host__ __device__ constexpr int comp_of(int j, int q)
{
    return V < 4 ? j * V + q : (j == 0 ? q : j == 1 ? 6 + q : (q < 2 ? 4 + q : 8 + q));
}

// Bytes from one right-hand side of a packed half field to the next: its 12
// component planes and a gap of RHS_GAP bytes; and 16-byte vectors from one
// plane to the next: Vh and a gap of PLANE_GAP (1 KiB).  Where Vh * 16 is a
// multiple of a large power of two (1 MiB for FP64 at 16^3 x 32) the planes of
// every right-hand side would all start at multiples of it.  Across right-hand
// sides that puts the few a hopping launch has in flight into the same L2
// sets, where they evict each other's neighbour spinors: with the RHS gap the
// plain FP64 hop of 288 right-hand sides at 16^3 x 32 fetched 1.66x instead of
// 1.71x its input bytes and took 1797 instead of 1877 us (a gap of 16.5 KiB:
// 1843 us).  The plane gap does not change the bytes fetched but took the same
// launch from 1786-1829 to 1737-1751 us (192 vectors: 1764-1786 us); the
// concurrent streams of one right-hand side's planes then no longer start at
// one offset modulo 1 MiB.
constexpr int64_t RHS_GAP = 1024;
#ifndef PLANE_GAP
#define PLANE_GAP 64
#endif
__host__ __device__ constexpr int64_t plane_stride(int64_t Vh) { return Vh + PLANE_GAP; }
__host__ __device__ constexpr int64_t rhs_stride_bytes(int64_t Vh, int64_t elem)
{
    return 12 * elem * plane_stride(Vh) + RHS_GAP;
}

template <typename S>
__device__ __forceinline__ const char *spinor_base(const Field &f, int64_t Vh, int rhs)
{
    return static_cast<const char *>(f.d) + (int64_t)rhs * rhs_stride_bytes(Vh, sizeof(typename Fmt<S>::E));
}

// NT: non-temporal loads (data the kernel reads once)
template <typename S, bool NT = false>
__device__ __forceinline__ void load_spinor(const Field &f, int64_t Vh, int rhs, int64_t cb,
                                            cx<typename Fmt<S>::R> v[12])
{
    using F = Fmt<S>;
    using R = typename F::R;
    using U4 = unsigned __attribute__((ext_vector_type(4)));
    constexpr int V = F::VEC;
    const uint4 *p = reinterpret_cast<const uint4 *>(spinor_base<S>(f, Vh, rhs));
#pragma unroll
    for (int j = 0; j < 12 / V; ++j) {
        uint4 q;
        if constexpr (NT) {
            const U4 raw = __builtin_nontemporal_load(reinterpret_cast<const U4 *>(p) + ((int64_t)j * plane_stride(Vh) + cb));
            __builtin_memcpy(&q, &raw, 16);
        } else {
            q = p[(int64_t)j * plane_stride(Vh) + cb];
        }
        cx<R> t[V];
        F::unpack(q, t);
#pragma unroll
        for (int k = 0; k < V; ++k) v[comp_of<V>(j, k)] = t[k];
    }
    if constexpr (F::scaled) {
        R s = NT ? __builtin_nontemporal_load(f.nrm + (int64_t)rhs * Vh + cb) : f.nrm[(int64_t)rhs * Vh + cb];
#pragma unroll
        for (int e = 0; e < 12; ++e) v[e] = s * v[e];
    }
}

// One spin pair of a stored spinor into v[0..5]: H = 0 the upper pair
// (components 0-5), H = 1 the lower pair (6-11).
template <typename S, int H>
__device__ __forceinline__ void load_half(const Field &f, int64_t Vh, int rhs, int64_t cb,
                                          cx<typename Fmt<S>::R> v[6])
{
    using F = Fmt<S>;
    using R = typename F::R;
    constexpr int V = F::VEC;
    const char *base = spinor_base<S>(f, Vh, rhs);
    const uint4 *p = reinterpret_cast<const uint4 *>(base);
    if constexpr (V == 4) {
        F::unpack(p[(int64_t)H * plane_stride(Vh) + cb], v);
        F::unpack2(reinterpret_cast<const uint2 *>(base)[(2 * plane_stride(Vh) + cb) * 2 + H], v + 4);
    } else {
#pragma unroll
        for (int j = 0; j < 6 / V; ++j) F::unpack(p[(int64_t)(H * 6 / V + j) * plane_stride(Vh) + cb], v + j * V);
    }
    if constexpr (F::scaled) {
        const R s = f.nrm[(int64_t)rhs * Vh + cb];
#pragma unroll
        for (int e = 0; e < 6; ++e) v[e] = s * v[e];
    }
}

// One right-hand side's half-spinor field as a buffer resource (its 12/VEC
// vectors of 16 bytes per site, vector j of site cb at byte (j Vp + cb) 16
// with Vp = plane_stride(Vh)).  A neighbour's loads then share one per-site
// byte offset in a VGPR and take the vector offset j Vp 16 from a scalar
// register: no 64-bit address arithmetic per load.  Requires
// 12 Vp sizeof(E) < 2^31 (checked by the launcher).  Reads past the resource
// return zero instead of faulting.
template <typename S>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t spinor_rsrc(const Field &f, int Vh, int rhs)
{
    const int bytes = 12 * (int)plane_stride(Vh) * (int)sizeof(typename Fmt<S>::E);
    char *base = static_cast<char *>(f.d) + (int64_t)rhs * rhs_stride_bytes(Vh, sizeof(typename Fmt<S>::E));
    // word 3: 32-bit data format, the value raw buffer loads use on this family
    return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, bytes, 0x00020000);
}

template <typename S>
__device__ __forceinline__ float load_scale_rsrc(const Field &f, int Vh, int rhs, int cb)
{
    const __amdgpu_buffer_rsrc_t rn =
        __builtin_amdgcn_make_buffer_rsrc(f.nrm + (int64_t)rhs * Vh, (short)0, Vh * 4, 0x00020000);
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rn, cb * 4, 0, 0));
}

// AUX: the loads' cache policy (0 = default; 2 = non-temporal, for data read
// once, so that it does not displace reused lines in L2).
template <typename S, int AUX = 0>
__device__ __forceinline__ void load_spinor_rsrc(__amdgpu_buffer_rsrc_t rs, const Field &f, int Vh, int rhs, int cb,
                                                 cx<typename Fmt<S>::R> v[12])
{
    using F = Fmt<S>;
    using R = typename F::R;
    constexpr int V = F::VEC;
    const int voff = cb * 16;
#pragma unroll
    for (int j = 0; j < 12 / V; ++j) {
        const auto raw = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, j * (int)plane_stride(Vh) * 16, AUX);
        uint4 q;
        __builtin_memcpy(&q, &raw, 16);
        cx<R> t[V];
        F::unpack(q, t);
#pragma unroll
        for (int k = 0; k < V; ++k) v[comp_of<V>(j, k)] = t[k];
    }
    if constexpr (F::scaled) {
        const R s = load_scale_rsrc<S>(f, Vh, rhs, cb);
#pragma unroll
        for (int e = 0; e < 12; ++e) v[e] = s * v[e];
    }
}

// One spin pair (H as load_half) through a buffer resource.
template <typename S, int H, int AUX = 0>
__device__ __forceinline__ void load_half_rsrc(__amdgpu_buffer_rsrc_t rs, const Field &f, int Vh, int rhs, int cb,
                                               cx<typename Fmt<S>::R> v[6])
{
    using F = Fmt<S>;
    using R = typename F::R;
    constexpr int V = F::VEC;
    const int voff = cb * 16;
    if constexpr (V == 4) {
        const auto raw = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, H * (int)plane_stride(Vh) * 16, AUX);
        uint4 q;
        __builtin_memcpy(&q, &raw, 16);
        F::unpack(q, v);
        const auto raw2 = __builtin_amdgcn_raw_buffer_load_b64(rs, voff + 8 * H, 2 * (int)plane_stride(Vh) * 16, AUX);
        uint2 q2;
        __builtin_memcpy(&q2, &raw2, 8);
        F::unpack2(q2, v + 4);
    } else {
#pragma unroll
        for (int j = 0; j < 6 / V; ++j) {
            const auto raw =
                __builtin_amdgcn_raw_buffer_load_b128(rs, voff, (H * 6 / V + j) * (int)plane_stride(Vh) * 16, AUX);
            uint4 q;
            __builtin_memcpy(&q, &raw, 16);
            F::unpack(q, v + j * V);
        }
    }
    if constexpr (F::scaled) {
        const R s = load_scale_rsrc<S>(f, Vh, rhs, cb);
#pragma unroll
        for (int e = 0; e < 6; ++e) v[e] = s * v[e];
    }
}

// NT: non-temporal stores (written once, not read again by this launch: they
// need not displace the lines the launch reuses in L2)
template <typename S, bool NT = false>
__device__ __forceinline__ void store_spinor(const Field &f, int64_t Vh, int rhs, int64_t cb,
                                             const cx<typename Fmt<S>::R> v[12])
{
    using F = Fmt<S>;
    using R = typename F::R;
    using U4 = unsigned __attribute__((ext_vector_type(4)));
    constexpr int V = F::VEC;
    uint4 *p = reinterpret_cast<uint4 *>(const_cast<char *>(spinor_base<S>(f, Vh, rhs)));
    auto put = [&](int j, const cx<R> *w) {
        cx<R> t[V];
#pragma unroll
        for (int k = 0; k < V; ++k) t[k] = w[comp_of<V>(j, k)];
        const uint4 q = F::pack(t);
        const int64_t k = (int64_t)j * plane_stride(Vh) + cb;
        if constexpr (NT) {
            U4 raw;
            __builtin_memcpy(&raw, &q, 16);
            __builtin_nontemporal_store(raw, reinterpret_cast<U4 *>(p) + k);
        } else {
            p[k] = q;
        }
    };
    if constexpr (F::scaled) {
        R m = 0;
#pragma unroll
        for (int e = 0; e < 12; ++e) m = fmaxf(m, fmaxf(fabsf(v[e].re), fabsf(v[e].im)));
        if constexpr (NT)
            __builtin_nontemporal_store(m, f.nrm + (int64_t)rhs * Vh + cb);
        else
            f.nrm[(int64_t)rhs * Vh + cb] = m;
        R inv = m > 0 ? R(1) / m : R(0);
        cx<R> w[12];
#pragma unroll
        for (int e = 0; e < 12; ++e) w[e] = inv * v[e];
#pragma unroll
        for (int j = 0; j < 12 / V; ++j) put(j, w);
    } else {
#pragma unroll
        for (int j = 0; j < 12 / V; ++j) put(j, v);
    }
}

// Link field of one precision: [4][2][NE][Vh].
template <typename S, int NE>
__device__ __forceinline__ void load_link(const void *links, int64_t Vh, int mu, int par, int64_t cb,
                                          cx<typename Fmt<S>::R> u[9])
{
    using F = Fmt<S>;
    const typename F::E *p = static_cast<const typename F::E *>(links) + ((int64_t)(mu * 2 + par) * NE) * Vh + cb;
#pragma unroll
    for (int e = 0; e < NE; ++e) u[e] = F::ld(p, e * Vh);
    if constexpr (NE == 6) {
        // third row = conj(row0 x row1) of a special-unitary matrix
        u[6] = conj(u[1] * u[5] - u[2] * u[4]);
        u[7] = conj(u[2] * u[3] - u[0] * u[5]);
        u[8] = conj(u[0] * u[4] - u[1] * u[3]);
    }
}

// ---------------------------------------------------------------- geometry

struct Geom {
    int X, Y, Z, T;  // full extents
    int Xh;          // X / 2
    int Vh;          // sites per parity
    int sY, sZ, sT;  // checkerboard strides of y, z, t: Xh, Xh*Y, Xh*Y*Z
    int tap;         // antiperiodic time boundary
};

struct Site {
    int x, y, z, t;
};

// coordinates of checkerboard site cb of parity p
__device__ __forceinline__ Site decode(const Geom &g, int cb, int p)
{
    Site s;
    int r = cb / g.Xh;
    int k = cb - r * g.Xh;
    int r2 = r / g.Y;
    s.y = r - r2 * g.Y;
    s.t = r2 / g.Z;
    s.z = r2 - s.t * g.Z;
    s.x = 2 * k + ((p + s.y + s.z + s.t) & 1);
    return s;
}

// ---------------------------------------------------------------- reductions

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Deterministic block sum of N values per thread; result valid in thread 0.
// scratch: __shared__ double[N * (blockDim/64)].
template <int N>
__device__ __forceinline__ void block_sum(double v[N], double *scratch)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < N; ++k) scratch[wid * N + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            double s = 0;
            for (int w = 0; w < nw; ++w) s += scratch[w * N + k];
            v[k] = s;
        }
    }
}

// ---------------------------------------------------------------- work distribution

// A launch covers up to MAXSEG segments (lattices of a batch, each with its
// own operands); prefix[s] is the first work item of segment s and
// prefix[n] the total.
constexpr int MAXSEG = 4;
template <typename A>
struct Segs {
    int n;
    int prefix[MAXSEG + 1];
    A a[MAXSEG];
};

// Visit the work items of this block.  The hardware hands consecutive
// workgroups to the 8 XCDs in turn; items are dealt out so that the blocks of
// one XCD walk one contiguous chunk of the item range, which keeps the
// neighbour sites a block gathers in that XCD's L2.  The grid is either one
// block per item or a multiple of 8 blocks (persistent: each block loops).
template <typename A, typename F>
__device__ __forceinline__ void for_each_item(const Segs<A> &B, F &&f)
{
    const int total = B.prefix[B.n];
    const int nx = 8, P = gridDim.x;
    const int xcd = blockIdx.x % nx, j = blockIdx.x / nx;
    const int nbx = P / nx + (xcd < P % nx ? 1 : 0);
    const int q = total / nx, rem = total % nx;
    const int start = xcd * q + min(xcd, rem), cnt = q + (xcd < rem ? 1 : 0);
    for (int i = j; i < cnt; i += nbx) {
        const int item = start + i;
        int s = 0;
        while (s + 1 < B.n && item >= B.prefix[s + 1]) ++s;
        f(B.a[s], item - B.prefix[s]);
    }
}

}  // namespace dl
