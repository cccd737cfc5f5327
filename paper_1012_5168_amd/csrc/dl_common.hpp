// dl_common.hpp -- device-side building blocks shared by the HIP kernels:
// complex arithmetic, storage formats of spinor and link fields, even-odd
// site geometry, wavefront reductions and the XCD-aware block order.
//
// Device layouts (private to the library):
//   half-spinor field of one parity, one right-hand side: 12 complex
//   components (spin-major, then colour) stored structure-of-arrays in
//   16-byte vectors of VEC consecutive components (VEC = 1 for FP64, 2 for
//   FP32, 4 for FP16 / BF16): component e of checkerboard site cb at element
//   [(e / VEC) * Vh + cb] * VEC + e % VEC, so one lane's 16-byte load brings
//   VEC components and a wavefront's load covers 64 consecutive sites; nrhs
//   fields follow each other with stride 12 * Vh elements.  FP16 fields carry
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
    // the k-th 16-byte vector of VEC components
    __device__ static __forceinline__ void ldv(const E *p, int64_t k, cx<double> v[1]) { v[0] = ld(p, k); }
    __device__ static __forceinline__ void stv(E *p, int64_t k, const cx<double> v[1]) { st(p, k, v[0]); }
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
    __device__ static __forceinline__ void ldv(const E *p, int64_t k, cx<float> v[2])
    {
        const float4 q = reinterpret_cast<const float4 *>(p)[k];
        v[0] = {q.x, q.y};
        v[1] = {q.z, q.w};
    }
    __device__ static __forceinline__ void stv(E *p, int64_t k, const cx<float> v[2])
    {
        reinterpret_cast<float4 *>(p)[k] = make_float4(v[0].re, v[0].im, v[1].re, v[1].im);
    }
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
__device__ __forceinline__ void ldv16(const H2 *p, int64_t k, cx<float> v[4], CVT cvt)
{
    unpack16<H2>(reinterpret_cast<const uint4 *>(p)[k], v, cvt);
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
template <typename H2, typename CVT>
__device__ __forceinline__ void stv16(H2 *p, int64_t k, const cx<float> v[4], CVT cvt)
{
    reinterpret_cast<uint4 *>(p)[k] = pack16<H2>(v, cvt);
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
    __device__ static __forceinline__ void ldv(const E *p, int64_t k, cx<float> v[4])
    {
        ldv16(p, k, v, [](E h) { return __half22float2(h); });
    }
    __device__ static __forceinline__ void stv(E *p, int64_t k, const cx<float> v[4])
    {
        stv16(p, k, v, [](float2 f) { return __float22half2_rn(f); });
    }
    __device__ static __forceinline__ void unpack(const uint4 &q, cx<float> v[4])
    {
        unpack16<E>(q, v, [](E h) { return __half22float2(h); });
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
    __device__ static __forceinline__ void ldv(const E *p, int64_t k, cx<float> v[4])
    {
        ldv16(p, k, v, [](E h) { return __bfloat1622float2(h); });
    }
    __device__ static __forceinline__ void stv(E *p, int64_t k, const cx<float> v[4])
    {
        stv16(p, k, v, [](float2 f) { return __float22bfloat162_rn(f); });
    }
    __device__ static __forceinline__ void unpack(const uint4 &q, cx<float> v[4])
    {
        unpack16<E>(q, v, [](E h) { return __bfloat1622float2(h); });
    }
    __device__ static __forceinline__ uint4 pack(const cx<float> v[4])
    {
        return pack16<E>(v, [](float2 f) { return __float22bfloat162_rn(f); });
    }
};

// A set of nrhs half-spinor fields of one parity.
struct Field {
    void *d;       // [nrhs][12][Vh] packed complex of the storage type
    float *nrm;    // [nrhs][Vh] per-site scale (FP16 only, else null)
};

// NT: non-temporal loads (data the kernel reads once)
template <typename S, bool NT = false>
__device__ __forceinline__ void load_spinor(const Field &f, int64_t Vh, int rhs, int64_t cb,
                                            cx<typename Fmt<S>::R> v[12])
{
    using F = Fmt<S>;
    using R = typename F::R;
    constexpr int V = F::VEC;
    const typename F::E *p = static_cast<const typename F::E *>(f.d) + (int64_t)rhs * 12 * Vh;
#pragma unroll
    for (int j = 0; j < 12 / V; ++j) {
        if constexpr (NT) {
            using U4 = unsigned __attribute__((ext_vector_type(4)));
            const U4 raw = __builtin_nontemporal_load(reinterpret_cast<const U4 *>(p) + ((int64_t)j * Vh + cb));
            uint4 q;
            __builtin_memcpy(&q, &raw, 16);
            F::unpack(q, v + j * V);
        } else {
            F::ldv(p, (int64_t)j * Vh + cb, v + j * V);
        }
    }
    if constexpr (F::scaled) {
        R s = NT ? __builtin_nontemporal_load(f.nrm + (int64_t)rhs * Vh + cb) : f.nrm[(int64_t)rhs * Vh + cb];
#pragma unroll
        for (int e = 0; e < 12; ++e) v[e] = s * v[e];
    }
}

// One right-hand side's half-spinor field as a buffer resource (its 12/VEC
// vectors of 16 bytes per site, vector j of site cb at byte (j Vh + cb) 16).
// A neighbour's loads then share one per-site byte offset in a VGPR and take
// the vector offset j Vh 16 from a scalar register: no 64-bit address
// arithmetic per load.  Requires 12 Vh sizeof(E) < 2^31 (checked by the
// launcher).  Reads past the resource return zero instead of faulting.
template <typename S>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t spinor_rsrc(const Field &f, int Vh, int rhs)
{
    const int bytes = 12 * Vh * (int)sizeof(typename Fmt<S>::E);
    char *base = static_cast<char *>(f.d) + (int64_t)rhs * bytes;
    // word 3: 32-bit data format, the value raw buffer loads use on this family
    return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, bytes, 0x00020000);
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
        const auto raw = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, j * Vh * 16, AUX);
        uint4 q;
        __builtin_memcpy(&q, &raw, 16);
        F::unpack(q, v + j * V);
    }
    if constexpr (F::scaled) {
        const __amdgpu_buffer_rsrc_t rn =
            __builtin_amdgcn_make_buffer_rsrc(f.nrm + (int64_t)rhs * Vh, (short)0, Vh * 4, 0x00020000);
        R s = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rn, cb * 4, 0, 0));
#pragma unroll
        for (int e = 0; e < 12; ++e) v[e] = s * v[e];
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
    typename F::E *p = static_cast<typename F::E *>(f.d) + (int64_t)rhs * 12 * Vh;
    auto put = [&](int64_t k, const cx<R> *w) {
        if constexpr (NT) {
            const uint4 q = F::pack(w);
            U4 raw;
            __builtin_memcpy(&raw, &q, 16);
            __builtin_nontemporal_store(raw, reinterpret_cast<U4 *>(p) + k);
        } else {
            F::stv(p, k, w);
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
        for (int j = 0; j < 12 / V; ++j) put((int64_t)j * Vh + cb, w + j * V);
    } else {
#pragma unroll
        for (int j = 0; j < 12 / V; ++j) put((int64_t)j * Vh + cb, v + j * V);
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
