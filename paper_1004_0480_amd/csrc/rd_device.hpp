// rd_device.hpp -- device code of the MI355X (gfx950) reaction-diffusion stepper.
//
// One explicit method-of-lines step (section 2, Eq. (5)):
//     c_s' = c_s + dt * ( L_s + A_s + R_s(c) + E_s )
// with L_s the 7-point Laplacian (per-axis coefficients), A_s first-order
// upwind advection, R_s the reaction at the old time level and E_s point
// sources.  Boundary values are virtual ghosts resolved while loading
// (section 4.1 sets them before each step; here they never touch memory).
//
// Every kernel variant funnels each cell through the same __device__ cell
// functions below, written with explicit fmaf and compiled with
// -ffp-contract=off, so all plans produce bitwise-identical fields.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace rdk {

enum { BC_MIRROR = 0, BC_PERIODIC = 1, BC_GHOST = 2, BC_HELD = 3 };

constexpr int MAXF = 5;          // stencil fields: up to 4 species + mu
constexpr int SLACK = 1024;      // elements after each buffer: overshoot of the widest tile

#ifndef RD_NT_STORE
#define RD_NT_STORE 0
#endif

// Step clock of a model with a time-dependent wind: the step index n of the
// state it belongs to and u_z(t_n)/h.  A grid keeps two, one per buffer
// parity; the step reading one writes the other.
struct StepClock {
    long long n;
    float uzh;
    int pad;
};

struct StepArgs {
    int nx, ny, nz;
    int pitch;                    // elements per padded row (multiple of 64)
    long long plane;              // elements per plane = pitch * ny
    const void* in[MAXF];         // fields read with the stencil
    void* out[MAXF];              // fields written
    float kx[MAXF], ky[MAXF], kz[MAXF];   // K_{f,d} / h^2
    float kc[MAXF];               // 2 (kx + ky + kz), formed once on the host
    int bck[MAXF][6];             // boundary kind per field and face
    float bcv[MAXF][6];           // boundary value per field and face
    int held[MAXF];               // bit f set: face f of field is BC_HELD
    int out_held[MAXF];           // held mask applied to output o (its field o)
    float dt;
    float p[8];                   // model constants (see the models)
    const float* wind_h;          // u(z)/h per z plane (pollutant)
    const int* src_row;           // nz*ny+1 offsets of the row-sorted sources
    const int* src_x;             // x of each source
    const int* src_sp;            // species of each source
    const float* src_rate;        // emission rate (duplicates merged)
    int sp0;                      // species of field 0 (source species are global)
    int s19;                      // 19-point Laplacian: kx = ky = kz = K/(6h^2)
    int tiles_x, tiles_y, chunks_z, cz;   // tiled decomposition
    int zfast;                    // slab enumeration: z chunk fastest
    // time-dependent wind (atmospheric model): u_z(t) = wamp sin(t / wper)
    // (wamp when wper = 0), t = t0 + n dt64
    const StepClock* clk_in;      // clock of this step's input state
    StepClock* clk_out;           // clock of its output state
    int clk_pass;                 // this pass advances the clock
    double t0, dt64, wamp, wper, inv_h;
    // stochastic rounding of BF16 stores: on/off, generator key (seed)
    int sr;
    unsigned sr_key;
    // Runge-Kutta stage: each stored state value v becomes b + w (v - b),
    // b = rk_base[s] at the same element (w = 0: a plain Euler step)
    const void* rk_base[MAXF];
    float rk_w;
};

// How a model's cell function gets its per-plane wind argument.
enum { WIND_NONE = 0, WIND_PLANE = 1, WIND_CLOCK = 2 };

// Tile coordinates of logical tile t: x, then y, then z chunk, or (zfast) z
// chunk, then x, then y.
struct TileXYZ { int x, y, z; };
__device__ __forceinline__ TileXYZ tile_coords(const StepArgs& a, int t) {
    if (a.zfast) {
        const int tz = t % a.chunks_z, r = t / a.chunks_z;
        return TileXYZ{r % a.tiles_x, r / a.tiles_x, tz};
    }
    const int tx = t % a.tiles_x, r = t / a.tiles_x;
    return TileXYZ{tx, r % a.tiles_y, r / a.tiles_y};
}

// --------------------------------------------------------------- storage

struct StF32 {
    using T = float;
    static __device__ __forceinline__ float up(T v) { return v; }
    static __device__ __forceinline__ T down(float v) { return v; }
};

typedef float rd_f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 rd_bf16x2 __attribute__((ext_vector_type(2)));

struct StBF16 {
    using T = uint16_t;
    static __device__ __forceinline__ float up(T v) { return __uint_as_float(uint32_t(v) << 16); }
    // round to nearest even (the hardware conversion); NaN stays NaN
    static __device__ __forceinline__ T down(float f) {
        const __bf16 b = (__bf16)f;
        T v;
        __builtin_memcpy(&v, &b, 2);
        return v;
    }
    // two values in one packed conversion, first value in the low half
    static __device__ __forceinline__ uint32_t down2(float f0, float f1) {
        rd_f32x2 x;
        x.x = f0;
        x.y = f1;
        const rd_bf16x2 b = __builtin_convertvector(x, rd_bf16x2);
        uint32_t v;
        __builtin_memcpy(&v, &b, 4);
        return v;
    }
};

struct StF16 {
    using T = uint16_t;
    static __device__ __forceinline__ float up(T v) {
        _Float16 h;
        __builtin_memcpy(&h, &v, 2);
        return float(h);
    }
    static __device__ __forceinline__ T down(float f) {
        _Float16 h = _Float16(f);          // v_cvt_f16_f32: round to nearest even
        T v;
        __builtin_memcpy(&v, &h, 2);
        return v;
    }
};

// FP64 as a transfer type only (rounded to FP32 first, then to storage).
struct StF64 {
    using T = double;
    static __device__ __forceinline__ float up(T v) { return float(v); }
};

// Field and table pointers reach the kernels inside the argument block in
// device memory, so the compiler sees generic pointers and would emit flat
// accesses, which also count against the LDS / scalar-load counter: every
// LDS exchange or scalar load would then wait for all loads in flight.  They
// always point to global memory; these casts say so.  (The host pass of the
// compiler only parses this code; it gets no address space.)
#ifdef __HIP_DEVICE_COMPILE__
#define RD_GLOBAL __attribute__((address_space(1)))
#define RD_CONST __attribute__((address_space(4)))
#define RD_LDS __attribute__((address_space(3)))
#else
#define RD_GLOBAL
#define RD_CONST
#define RD_LDS
#endif
template <typename T>
__device__ __forceinline__ const RD_GLOBAL T* gload_ptr(const void* p) {
    return (const RD_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ RD_GLOBAL T* gstore_ptr(void* p) {
    return (RD_GLOBAL T*)p;
}
// Tables that no thread of the running launch writes -- the clock of the
// step's input state, the wind profile, the source lists -- are read as
// constant memory: a uniform index then becomes a scalar load, and the
// compiler may reuse one load across the launch's stores instead of issuing
// a vector load (and a wait on every store in flight) at each use.
template <typename T>
__device__ __forceinline__ const RD_CONST T* cload_ptr(const void* p) {
    return (const RD_CONST T*)p;
}

// The LDS-ring kernels address their rings through LDS pointers taken from
// the __shared__ arrays themselves, never through generic pointers.
typedef float lds_v4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void lds_ld4(const RD_LDS float* p, float (&o)[4]) {
    const lds_v4 t = *(const RD_LDS lds_v4*)p;
    o[0] = t.x; o[1] = t.y; o[2] = t.z; o[3] = t.w;
}
__device__ __forceinline__ void lds_st4(RD_LDS float* p, float x, float y, float z, float w) {
    lds_v4 t;
    t.x = x; t.y = y; t.z = z; t.w = w;
    *(RD_LDS lds_v4*)p = t;
}

// N contiguous elements of type T as one naturally aligned access.
template <typename T, int N> struct alignas(sizeof(T) * N) Vec { T v[N]; };

template <class S, int VX>
__device__ __forceinline__ void load_vec(const void* base, long long idx, float (&o)[VX]) {
    using T = typename S::T;
    const Vec<T, VX> r = *(const RD_GLOBAL Vec<T, VX>*)(gload_ptr<T>(base) + idx);
#pragma unroll
    for (int i = 0; i < VX; ++i) o[i] = S::up(r.v[i]);
}

template <class S, int VX>
__device__ __forceinline__ void store_vec_at(RD_GLOBAL typename S::T* dst, const float (&o)[VX]) {
    using T = typename S::T;
    Vec<T, VX> r;
    if constexpr (std::is_same_v<S, StBF16> && VX % 2 == 0) {
        // pairs through the packed conversion
#pragma unroll
        for (int i = 0; i < VX; i += 2) {
            const uint32_t p = StBF16::down2(o[i], o[i + 1]);
            r.v[i] = T(p & 0xffffu);
            r.v[i + 1] = T(p >> 16);
        }
    } else {
#pragma unroll
        for (int i = 0; i < VX; ++i) r.v[i] = S::down(o[i]);
    }
#if RD_NT_STORE
    // streaming store: the next step reads these values from HBM anyway
    if constexpr (sizeof(r) == 16) {
        typedef unsigned v4u __attribute__((ext_vector_type(4)));
        __builtin_nontemporal_store(*reinterpret_cast<const v4u*>(&r), (RD_GLOBAL v4u*)dst);
    } else if constexpr (sizeof(r) == 8) {
        typedef unsigned v2u __attribute__((ext_vector_type(2)));
        __builtin_nontemporal_store(*reinterpret_cast<const v2u*>(&r), (RD_GLOBAL v2u*)dst);
    } else if constexpr (sizeof(r) == 4) {
        __builtin_nontemporal_store(*reinterpret_cast<const unsigned*>(&r), (RD_GLOBAL unsigned*)dst);
    } else {
        *(RD_GLOBAL Vec<T, VX>*)dst = r;
    }
#else
    *(RD_GLOBAL Vec<T, VX>*)dst = r;
#endif
}

template <class S, int VX>
__device__ __forceinline__ void store_vec(void* base, long long idx, const float (&o)[VX]) {
    store_vec_at<S, VX>(gstore_ptr<typename S::T>(base) + idx, o);
}

template <class S>
__device__ __forceinline__ float load1(const void* base, long long idx) {
    return S::up(gload_ptr<typename S::T>(base)[idx]);
}

// ---- stochastic rounding of BF16 stores --------------------------------
//
// Counter-based random bits: Philox-2x32 with 10 rounds (Salmon, Moraes,
// Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11): each
// round multiplies the first counter word by 0xD256D193, the new first word
// is the high half xor the key xor the second word, the new second word the
// low half, and the key is bumped by 0x9E3779B9.  One call gives 64 bits,
// which serve four stored elements: element e of a field (its dense index
// (z*ny + y)*nx + x) takes 16 bits of the output for counter (e/4, step
// index) and key (seed + species) -- bits 0-15 of the first word for e%4 = 0,
// 16-31 for 1, then the same halves of the second word for 2 and 3.
struct PhiloxOut { unsigned w0, w1; };

__device__ __forceinline__ PhiloxOut philox2x32_10(unsigned c0, unsigned c1, unsigned k) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // the whole 64-bit product in one multiply-add (v_mad_u64_u32)
        // rather than separate high and low multiplies
        const unsigned long long p = (unsigned long long)0xD256D193u * c0;
        c0 = unsigned(p >> 32) ^ k ^ c1;
        c1 = unsigned(p);
        k += 0x9E3779B9u;
    }
    return PhiloxOut{c0, c1};
}

__device__ __forceinline__ unsigned philox_bits16(const PhiloxOut& r, unsigned q) {
    const unsigned w = (q & 2u) ? r.w1 : r.w0;
    return (q & 1u) ? (w >> 16) : (w & 0xffffu);
}

// Stochastic rounding to BF16: add 16 random bits to the FP32 pattern and
// keep the high half, so the magnitude rounds up with probability (low 16
// bits) / 2^16 and the expected stored value is the FP32 one.  Infinities
// and NaN round as to nearest.
__device__ __forceinline__ uint16_t bf16_stochastic(float f, unsigned r16) {
    const unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) >= 0x7f800000u) return StBF16::down(f);
    return uint16_t((u + r16) >> 16);
}

// A Runge-Kutta stage's combination of an Euler result v with the state b
// at the same element: b + w (v - b), which keeps a held value exactly.
template <class S, int VX>
__device__ __forceinline__ void rk_blend(const StepArgs& a, int s, long long idx, float (&o)[VX]) {
    if (a.rk_w != 0.f) {
        float b[VX];
        load_vec<S, VX>(a.rk_base[s], idx, b);
#pragma unroll
        for (int i = 0; i < VX; ++i) o[i] = __fmaf_rn(a.rk_w, o[i] - b[i], b[i]);
    }
}

// Store VX output values of species s (of this pass) at row element x of
// row y, plane z, in the storage type (after a Runge-Kutta stage's
// combination), rounding stochastically when the grid asks for it.
template <class S, int VX>
__device__ __forceinline__ void store_field(const StepArgs& a, int s, int x, int y, int z, const float (&v)[VX]) {
    const long long idx = (long long)z * a.plane + (long long)y * a.pitch + x;
    float o[VX];
#pragma unroll
    for (int i = 0; i < VX; ++i) o[i] = v[i];
    rk_blend<S, VX>(a, s, idx, o);
    if constexpr (std::is_same_v<S, StBF16>) {
        if (a.sr) {
            const unsigned n = unsigned(cload_ptr<StepClock>(a.clk_in)->n);
            const unsigned key = a.sr_key + unsigned(a.sp0 + s);
            const unsigned long long e0 = ((unsigned long long)z * unsigned(a.ny) + unsigned(y)) * unsigned(a.nx) +
                                          unsigned(x);
            Vec<uint16_t, VX> w;
            // G elements starting at a multiple of G share one counter: then
            // the VX elements need exactly ceil(VX / 4) calls (the kernels
            // place a lane's cells at multiples of VX, so this holds whenever
            // the row length is a multiple of G)
            constexpr int G = VX >= 4 ? 4 : VX;
            if (G > 1 && VX % G == 0 && (unsigned(e0) & unsigned(G - 1)) == 0) {
                const unsigned c0 = unsigned(e0 >> 2);
#pragma unroll
                for (int g = 0; g < VX / G; ++g) {
                    const PhiloxOut r = philox2x32_10(c0 + unsigned(g * G / 4), n, key);
                    if constexpr (G == 4) {
                        w.v[4 * g + 0] = bf16_stochastic(o[4 * g + 0], r.w0 & 0xffffu);
                        w.v[4 * g + 1] = bf16_stochastic(o[4 * g + 1], r.w0 >> 16);
                        w.v[4 * g + 2] = bf16_stochastic(o[4 * g + 2], r.w1 & 0xffffu);
                        w.v[4 * g + 3] = bf16_stochastic(o[4 * g + 3], r.w1 >> 16);
                    } else {
                        const unsigned wd = (unsigned(e0) & 2u) ? r.w1 : r.w0;
                        w.v[0] = bf16_stochastic(o[0], wd & 0xffffu);
                        w.v[1] = bf16_stochastic(o[1], wd >> 16);
                    }
                }
            } else {
                // the VX elements span at most NR consecutive counters
                constexpr int NR = (VX + 6) / 4;
                const unsigned c_first = unsigned(e0 >> 2), c_last = unsigned((e0 + VX - 1) >> 2);
                PhiloxOut r[NR];
#pragma unroll
                for (int k = 0; k < NR; ++k) {
                    r[k] = PhiloxOut{0u, 0u};
                    if (c_first + unsigned(k) <= c_last) r[k] = philox2x32_10(c_first + unsigned(k), n, key);
                }
#pragma unroll
                for (int i = 0; i < VX; ++i) {
                    const unsigned long long e = e0 + unsigned(i);
                    const unsigned kk = unsigned(e >> 2) - c_first;
                    PhiloxOut ri = r[0];
#pragma unroll
                    for (int k = 1; k < NR; ++k) ri = kk == unsigned(k) ? r[k] : ri;
                    w.v[i] = bf16_stochastic(o[i], philox_bits16(ri, unsigned(e) & 3u));
                }
            }
            *(RD_GLOBAL Vec<uint16_t, VX>*)(gstore_ptr<uint16_t>(a.out[s]) + idx) = w;
            return;
        }
    }
    store_vec<S, VX>(a.out[s], idx, o);
}

// --------------------------------------------------------- cell arithmetic

struct Nb { float c, xm, xp, ym, yp, zm, zp; };

// sum_d K_d (c[+e_d] + c[-e_d] - 2c), K already divided by h^2
__device__ __forceinline__ float lap7(const Nb& n, float kx, float ky, float kz) {
    const float c2 = n.c + n.c;
    const float dx = (n.xm + n.xp) - c2;
    const float dy = (n.ym + n.yp) - c2;
    const float dz = (n.zm + n.zp) - c2;
    return __fmaf_rn(kx, dx, __fmaf_rn(ky, dy, kz * dz));
}

// The 19 points of Eqs. (3)-(4): the 7 above plus the twelve edge
// neighbours, carried as three partial sums that both kernel families form
// in the same order:
//   s   = (c[y-1] + c[y+1]) + (c[z-1] + c[z+1])            (the centre's cross)
//   sxm = the same cross sum one cell to the left (the four x- edges),
//   sxp = the same one cell to the right (the four x+ edges),
//   q   = (c[y-1,z-1] + c[y+1,z-1]) + (c[y-1,z+1] + c[y+1,z+1]).
// Beyond an x face every term of a cross sum follows the face rule of x, so
// sxm / sxp there are the cross sum at the mirrored or wrapped cell, or four
// times the face value.
struct Nb19 : Nb { float s, sxm, sxp, q; };

// K/(6h^2) * (-24 c + 2 * faces + edges), K/(6h^2) given (isotropic)
__device__ __forceinline__ float lap19(const Nb19& n, float k6) {
    const float faces = (n.xm + n.xp) + n.s;
    const float edges = (n.sxm + n.sxp) + n.q;
    return k6 * __fmaf_rn(-24.f, n.c, __fmaf_rn(2.f, faces, edges));
}

// The front model's 7-point form: the neighbour pairs weighted by their axis
// coefficients, less kc = 2 (kx + ky + kz) times the centre (7 operations
// against 10; every kernel of that model forms it so).
__device__ __forceinline__ float lap7s(const Nb& n, float kx, float ky, float kz, float kc) {
    return __fmaf_rn(-kc, n.c, __fmaf_rn(kx, n.xm + n.xp, __fmaf_rn(ky, n.ym + n.yp, kz * (n.zm + n.zp))));
}
// (P: the step arguments, or any copy of their coefficients kx, ky, kz, kc)
template <class P>
__device__ __forceinline__ float lapf(const Nb& n, const P& a, int f) {
    return lap7s(n, a.kx[f], a.ky[f], a.kz[f], a.kc[f]);
}
template <class P>
__device__ __forceinline__ float lapf(const Nb19& n, const P& a, int f) { return lap19(n, a.kx[f]); }

// A per-lane copy of a uniform value: the copy lives in a VGPR for the whole
// z march, so the plane loops of the marching kernels issue no scalar reloads
// of the launch's constants (scalar loads share the LDS reads' wait counter,
// so each reload would also stall on every LDS read in flight) and the SGPRs
// stay free for the loop's own scalars.
__device__ __forceinline__ float vcopy(float x) {
#ifdef __HIP_DEVICE_COMPILE__
    float r;
    asm("v_mov_b32 %0, %1" : "=v"(r) : "s"(x));
    return r;
#else
    return x;
#endif
}

// The coefficients the cell functions read, under the step arguments' names
// (so the cell arithmetic takes either), copied once per wave.
struct CellConst {
    float kx[MAXF], ky[MAXF], kz[MAXF], kc[MAXF];
    float p[8];
    float dt;
    __device__ __forceinline__ explicit CellConst(const StepArgs& a) {
#pragma unroll
        for (int f = 0; f < MAXF; ++f) {
            kx[f] = vcopy(a.kx[f]);
            ky[f] = vcopy(a.ky[f]);
            kz[f] = vcopy(a.kz[f]);
            kc[f] = vcopy(a.kc[f]);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) p[i] = vcopy(a.p[i]);
        dt = vcopy(a.dt);
    }
};

// The Laplacian of a neighbourhood: 7-point (per-axis K/h^2) or 19-point
// (all three coefficients hold K/(6h^2)).
__device__ __forceinline__ float lap(const Nb& n, float kx, float ky, float kz) { return lap7(n, kx, ky, kz); }
__device__ __forceinline__ float lap(const Nb19& n, float kx, float, float) { return lap19(n, kx); }

// First-order upwind form of -u dc/dx along one axis, uh = u/h: the
// difference on the side the wind comes from, u (c[-1] - c) / h for u > 0
// and u (c - c[+1]) / h for u < 0.
__device__ __forceinline__ float upwind(float uh, float cm, float cp, float c, float rate) {
    return __fmaf_rn(uh, uh > 0.f ? cm - c : c - cp, rate);
}

// Pure diffusion of NS independent species (Table 1, first row).
template <int NS> struct Diffusion {
    static constexpr int NF = NS, NO = NS;
    static constexpr bool SOURCES = false;
    static constexpr int WIND = WIND_NONE;
    static __host__ __device__ constexpr bool f32_field(int) { return false; }
    static __host__ __device__ constexpr bool f32_out(int) { return false; }
    template <class NB, class P>
    static __device__ __forceinline__ void cell(const P& a, const NB (&n)[NF], float,
                                                bool, const float (&)[NO], float (&o)[NO]) {
#pragma unroll
        for (int s = 0; s < NS; ++s)
            o[s] = __fmaf_rn(a.dt, lap(n[s], a.kx[s], a.ky[s], a.kz[s]), n[s].c);
    }
};

// Brusselator activator-inhibitor kinetics: p[0]=a, p[1]=b, p[2]=-(b+1).
struct Brusselator {
    static constexpr int NF = 2, NO = 2;
    static constexpr bool SOURCES = false;
    static constexpr int WIND = WIND_NONE;
    static __host__ __device__ constexpr bool f32_field(int) { return false; }
    static __host__ __device__ constexpr bool f32_out(int) { return false; }
    template <class NB, class P>
    static __device__ __forceinline__ void cell(const P& a, const NB (&n)[2], float,
                                                bool, const float (&)[2], float (&o)[2]) {
        const float u = n[0].c, v = n[1].c;
        const float uuv = (u * u) * v;
        const float ru = __fmaf_rn(a.p[2], u, a.p[0] + uuv);   // a - (b+1) u + u^2 v
        const float rv = __fmaf_rn(a.p[1], u, -uuv);            // b u - u^2 v
        const float lu = lap(n[0], a.kx[0], a.ky[0], a.kz[0]);
        const float lv = lap(n[1], a.kx[1], a.ky[1], a.kz[1]);
        o[0] = __fmaf_rn(a.dt, lu + ru, u);
        o[1] = __fmaf_rn(a.dt, lv + rv, v);
    }
};

// Cahn-Hilliard first pass: mu = gamma C^3 - eps C - kappa Lap(C).
// Field 0 is C (its own faces); output 0 is mu in FP32.
// p[2]=kappa p[3]=eps p[4]=gamma; kx[0]=ky[0]=kz[0]=1/h^2.
struct ChemPotential {
    static constexpr int NF = 1, NO = 1;
    static constexpr bool SOURCES = false;
    static constexpr int WIND = WIND_NONE;
    static __host__ __device__ constexpr bool f32_field(int) { return false; }
    static __host__ __device__ constexpr bool f32_out(int) { return true; }
    // mu of a cell from C there and Lap(C) there (every kernel forms it so;
    // P: the step arguments or a copy of their parameters p)
    template <class P>
    static __device__ __forceinline__ float mu(const P& a, float c, float lc) {
        return __fmaf_rn(-a.p[2], lc, __fmaf_rn(a.p[4] * c, c * c, -(a.p[3] * c)));
    }
    template <class NB, class P>
    static __device__ __forceinline__ void cell(const P& a, const NB (&n)[1], float,
                                                bool, const float (&)[1], float (&o)[1]) {
        o[0] = mu(a, n[0].c, lapf(n[0], a, 0));
    }
};

// Front with precipitation: A + B -> C at rate k, redissolution A + C at
// rate k2 (removes A and C), C moves by M Lap(mu).
// Fields 0..2 = A, B, C (storage type), field 3 = mu (FP32, mirror faces).
// p[0]=k p[1]=M p[5]=k2; kx[3]=ky[3]=kz[3]=1/h^2.
struct FrontCH {
    static constexpr int NF = 4, NO = 3;
    static constexpr bool SOURCES = false;
    static constexpr int WIND = WIND_NONE;
    static __host__ __device__ constexpr bool f32_field(int f) { return f == 3; }
    static __host__ __device__ constexpr bool f32_out(int) { return false; }
    // the update from the cell's values and Laplacians; q = k2 A C (P: the
    // step arguments or a copy of their parameters p and dt)
    template <class P>
    static __device__ __forceinline__ void rates(const P& a, float A, float B, float C, float la, float lb,
                                                 float lc, float lmu, float q, float (&o)[3]) {
        const float r = (a.p[0] * A) * B;
        o[0] = __fmaf_rn(a.dt, (la - r) - q, A);
        o[1] = __fmaf_rn(a.dt, lb - r, B);
        o[2] = __fmaf_rn(a.dt, __fmaf_rn(a.p[1], lmu, lc + r) - q, C);
    }
    template <class NB, class P>
    static __device__ __forceinline__ void cell(const P& a, const NB (&n)[4], float,
                                                bool, const float (&)[3], float (&o)[3]) {
        const float A = n[0].c, B = n[1].c, C = n[2].c;
        const float q = (a.p[5] * A) * C;
        const float la = lapf(n[0], a, 0);
        const float lb = lapf(n[1], a, 1);
        const float lc = lapf(n[2], a, 2);
        const float lmu = lapf(n[3], a, 3);
        rates(a, A, B, C, la, lb, lc, lmu, q, o);
    }
};

// Advection-diffusion of NS pollutants: upwind wind along +x (u(z)/h given),
// first-order decay p[0], and (COUPLED) transfer p[1] from field 0 to field
// 1, plus point sources.  A step of more species runs as several passes over
// groups that share no term: the coupled pair, then the others.
template <int NS, bool COUPLED> struct Pollutant {
    static constexpr int NF = NS, NO = NS;
    static constexpr bool SOURCES = true;
    static constexpr int WIND = WIND_PLANE;
    static __host__ __device__ constexpr bool f32_field(int) { return false; }
    static __host__ __device__ constexpr bool f32_out(int) { return false; }
    template <class NB, class P>
    static __device__ __forceinline__ void cell(const P& a, const NB (&n)[NF], float uh,
                                                bool has_e, const float (&e)[NO], float (&o)[NO]) {
        const float c0 = n[0].c;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const float c = n[s].c;
            float rate = lap(n[s], a.kx[s], a.ky[s], a.kz[s]);
            rate = __fmaf_rn(uh, n[s].xm - c, rate);       // -u (c_i - c_{i-1}) / h
            rate = __fmaf_rn(-a.p[0], c, rate);             // decay
            if (COUPLED && NS >= 2 && s == 0) rate = __fmaf_rn(-a.p[1], c0, rate);
            if (COUPLED && NS >= 2 && s == 1) rate = __fmaf_rn(a.p[1], c0, rate);
            if (has_e) rate = rate + e[s];
            o[s] = __fmaf_rn(a.dt, rate, c);
        }
    }
};

// Activator-inhibitor kinetics of Table 1 (second row):
// R_1 = c_1 - c_1^3 - c_2,  R_2 = gamma (c_1 - alpha c_2 - beta).
// p[0]=alpha p[1]=beta p[2]=gamma.
struct Turing {
    static constexpr int NF = 2, NO = 2;
    static constexpr bool SOURCES = false;
    static constexpr int WIND = WIND_NONE;
    static __host__ __device__ constexpr bool f32_field(int) { return false; }
    static __host__ __device__ constexpr bool f32_out(int) { return false; }
    template <class NB, class P>
    static __device__ __forceinline__ void cell(const P& a, const NB (&n)[2], float,
                                                bool, const float (&)[2], float (&o)[2]) {
        const float u = n[0].c, v = n[1].c;
        const float r1 = (u - (u * u) * u) - v;
        const float r2 = a.p[2] * (__fmaf_rn(-a.p[0], v, u) - a.p[1]);
        const float l1 = lap(n[0], a.kx[0], a.ky[0], a.kz[0]);
        const float l2 = lap(n[1], a.kx[1], a.ky[1], a.kz[1]);
        o[0] = __fmaf_rn(a.dt, l1 + r1, u);
        o[1] = __fmaf_rn(a.dt, l2 + r2, v);
    }
};

// Atmospheric advection-diffusion of NS independent species (Table 1, last
// row): a wind uniform in space, u_x and u_y fixed (p[0] = u_x/h, p[1] =
// u_y/h), u_z(t)/h from the step clock (the cell's wind argument), each
// axis upwinded by the sign of its component, plus point emissions.
template <int NS> struct Atmos {
    static constexpr int NF = NS, NO = NS;
    static constexpr bool SOURCES = true;
    static constexpr int WIND = WIND_CLOCK;
    static __host__ __device__ constexpr bool f32_field(int) { return false; }
    static __host__ __device__ constexpr bool f32_out(int) { return false; }
    template <class NB, class P>
    static __device__ __forceinline__ void cell(const P& a, const NB (&n)[NF], float uzh,
                                                bool has_e, const float (&e)[NO], float (&o)[NO]) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const float c = n[s].c;
            float rate = lap(n[s], a.kx[s], a.ky[s], a.kz[s]);
            rate = upwind(a.p[0], n[s].xm, n[s].xp, c, rate);
            rate = upwind(a.p[1], n[s].ym, n[s].yp, c, rate);
            rate = upwind(uzh, n[s].zm, n[s].zp, c, rate);
            if (has_e) rate = rate + e[s];
            o[s] = __fmaf_rn(a.dt, rate, c);
        }
    }
};

// The wind argument of a model's cell function on plane z.
template <class M>
__device__ __forceinline__ float plane_wind(const StepArgs& a, int z) {
    if constexpr (M::WIND == WIND_PLANE) return cload_ptr<float>(a.wind_h)[z];
    else if constexpr (M::WIND == WIND_CLOCK) return cload_ptr<StepClock>(a.clk_in)->uzh;
    else return 0.f;
}

// One thread of the clock pass writes the clock of the step's output state:
// n + 1 and u_z(t_{n+1})/h, in FP64 as the time is formed.
// The clock also counts steps for stochastic rounding.
template <class M>
__device__ __forceinline__ void tick_clock(const StepArgs& a, bool first_thread) {
    if (first_thread && a.clk_pass && (M::WIND == WIND_CLOCK || a.sr)) {
        const long long n = cload_ptr<StepClock>(a.clk_in)->n + 1;
        double u = 0.0;
        if constexpr (M::WIND == WIND_CLOCK) {
            const double t = a.t0 + double(n) * a.dt64;
            u = a.wper != 0.0 ? a.wamp * sin(t / a.wper) : a.wamp;
        }
        StepClock* out = gstore_ptr<StepClock>(a.clk_out);
        out->n = n;
        out->uzh = float(u * a.inv_h);
    }
}

// ------------------------------------------------------------ ghost logic

// The value one cell beyond index 0 / n-1 comes from (idx, rule, value) by
// the face rule; an in-range index on a held face reads the held value.
// cst: 0 = load from idx, 1 = held layer, 2 = fixed ghost beyond the face.
// A ghost beyond a face takes that face's rule before any held layer of
// another axis; held layers go by x-, x+, y-, y+, z-, z+.
enum { CST_NONE = 0, CST_HELD = 1, CST_GHOST = 2 };
struct Src { int idx; int cst; float v; };

__device__ __forceinline__ Src resolve_axis(int q, int n, int klo, int khi, float vlo, float vhi) {
    const bool lo = q < 0, hi = q >= n;
    const bool fixed_lo = klo == BC_GHOST || klo == BC_HELD;
    const bool fixed_hi = khi == BC_GHOST || khi == BC_HELD;
    int idx = q;
    idx = lo ? (klo == BC_PERIODIC ? n - 1 : 0) : idx;
    idx = hi ? ((q > n || khi != BC_PERIODIC) ? n - 1 : 0) : idx;   // beyond the ghost: unused
    const bool ghost = (lo && fixed_lo) || (hi && q == n && fixed_hi);
    float v = lo ? vlo : vhi;
    // a resolved in-range index on a held face reads the held value (lo first)
    const bool hlo = !ghost && idx == 0 && klo == BC_HELD;
    const bool hhi = !ghost && !hlo && idx == n - 1 && khi == BC_HELD;
    v = hlo ? vlo : (hhi ? vhi : v);
    return Src{idx, ghost ? CST_GHOST : (hlo || hhi) ? CST_HELD : CST_NONE, v};
}

// Value at a point whose three axes resolved to sx, sy, sz (at most one of
// them from outside the grid), given the value v loaded from the resolved
// address.
__device__ __forceinline__ float fixed_or(const Src& sx, const Src& sy, const Src& sz, float v) {
    return sx.cst == CST_GHOST ? sx.v : sy.cst == CST_GHOST ? sy.v : sz.cst == CST_GHOST ? sz.v
         : sx.cst ? sx.v : sy.cst ? sy.v : sz.cst ? sz.v : v;
}

// The 7 stencil values of field f around in-range (x, y, z).  Each axis is
// resolved by its face rules (the centre's resolution serves the two axes a
// neighbour does not move along), one load is made from every resolved
// (always valid) address, and a value fixed by a rule replaces it.  Written
// as value selects so that no address depends on the rules.
template <class S, bool S19>
__device__ __forceinline__ std::conditional_t<S19, Nb19, Nb> stencil(const StepArgs& a, int f, int x, int y, int z) {
    const int* k = a.bck[f];
    const float* v = a.bcv[f];
    const Src sx = resolve_axis(x, a.nx, k[0], k[1], v[0], v[1]);
    const Src sy = resolve_axis(y, a.ny, k[2], k[3], v[2], v[3]);
    const Src sz = resolve_axis(z, a.nz, k[4], k[5], v[4], v[5]);
    const Src xm = resolve_axis(x - 1, a.nx, k[0], k[1], v[0], v[1]);
    const Src xp = resolve_axis(x + 1, a.nx, k[0], k[1], v[0], v[1]);
    const Src ym = resolve_axis(y - 1, a.ny, k[2], k[3], v[2], v[3]);
    const Src yp = resolve_axis(y + 1, a.ny, k[2], k[3], v[2], v[3]);
    const Src zm = resolve_axis(z - 1, a.nz, k[4], k[5], v[4], v[5]);
    const Src zp = resolve_axis(z + 1, a.nz, k[4], k[5], v[4], v[5]);
    // an edge neighbour leaves along two axes: fixed_or takes the ghost of
    // the first of them (x, y, z), a mirror or periodic axis its resolved index
    auto at = [&](const Src& qx, const Src& qy, const Src& qz) __attribute__((always_inline)) {
        const float u = load1<S>(a.in[f], (long long)qz.idx * a.plane + (long long)qy.idx * a.pitch + qx.idx);
        return fixed_or(qx, qy, qz, u);
    };
    std::conditional_t<S19, Nb19, Nb> n;
    n.c = at(sx, sy, sz);
    n.xm = at(xm, sy, sz);
    n.xp = at(xp, sy, sz);
    n.ym = at(sx, ym, sz);
    n.yp = at(sx, yp, sz);
    n.zm = at(sx, sy, zm);
    n.zp = at(sx, sy, zp);
    if constexpr (S19) {
        n.s = (n.ym + n.yp) + (n.zm + n.zp);
        n.sxm = (at(xm, ym, sz) + at(xm, yp, sz)) + (at(xm, sy, zm) + at(xm, sy, zp));
        n.sxp = (at(xp, ym, sz) + at(xp, yp, sz)) + (at(xp, sy, zm) + at(xp, sy, zp));
        n.q = (at(sx, ym, zm) + at(sx, yp, zm)) + (at(sx, ym, zp) + at(sx, yp, zp));
    }
    return n;
}

// Merged emission rates of the cell at x of a row whose sources are
// [s0, s1); `any` is false if the cell has none.  Returned by value so the
// rates stay in registers.
template <int NO> struct Emission {
    float e[NO];
    bool any;
};

template <int NO>
__device__ __forceinline__ Emission<NO> cell_sources(const StepArgs& a, int x, int s0, int s1) {
    Emission<NO> r;
#pragma unroll
    for (int s = 0; s < NO; ++s) r.e[s] = 0.f;
    r.any = false;
    for (int q = s0; q < s1; ++q) {
        if (cload_ptr<int>(a.src_x)[q] == x) {
            const int sp = cload_ptr<int>(a.src_sp)[q];
            const float rate = cload_ptr<float>(a.src_rate)[q];
#pragma unroll
            for (int s = 0; s < NO; ++s) r.e[s] = sp - a.sp0 == s ? rate : r.e[s];
            r.any = true;
        }
    }
    return r;
}

// Output value of species s at (x, y, z): the held value on a held face, else
// v.  Takes and returns the value (not a reference) so that the choice stays
// a register select and the outputs never go through memory.
__device__ __forceinline__ float held_out(const StepArgs& a, int s, int x, int y, int z, float v) {
    const int hm = a.out_held[s];
    if (hm) {
        if ((hm & 32) && z == a.nz - 1) v = a.bcv[s][5];
        if ((hm & 16) && z == 0) v = a.bcv[s][4];
        if ((hm & 8) && y == a.ny - 1) v = a.bcv[s][3];
        if ((hm & 4) && y == 0) v = a.bcv[s][2];
        if ((hm & 2) && x == a.nx - 1) v = a.bcv[s][1];
        if ((hm & 1) && x == 0) v = a.bcv[s][0];
    }
    return v;
}

// ------------------------------------------------------------ direct kernel
// One thread per cell; all 7 (or 19) stencil points come through the cache.  The
// simple baseline the tiled plans are checked against bit for bit.

template <class M, class S, bool S19>
__global__ __launch_bounds__(256) void direct_kernel(const StepArgs* __restrict__ pa) {
    const StepArgs& a = *pa;
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int z = blockIdx.z;
    tick_clock<M>(a, (blockIdx.x | blockIdx.y | blockIdx.z | threadIdx.x) == 0);
    if (x >= a.nx || y >= a.ny) return;
    std::conditional_t<S19, Nb19, Nb> n[M::NF];
#pragma unroll
    for (int f = 0; f < M::NF; ++f)
        n[f] = M::f32_field(f) ? stencil<StF32, S19>(a, f, x, y, z) : stencil<S, S19>(a, f, x, y, z);
    Emission<M::NO> em{};
    if (M::SOURCES) {
        const int r = z * a.ny + y;
        em = cell_sources<M::NO>(a, x, cload_ptr<int>(a.src_row)[r], cload_ptr<int>(a.src_row)[r + 1]);
    }
    const float uh = plane_wind<M>(a, z);
    float o[M::NO];
    M::cell(a, n, uh, em.any, em.e, o);
    const long long idx = (long long)z * a.plane + (long long)y * a.pitch + x;
#pragma unroll
    for (int s = 0; s < M::NO; ++s) {
        const float v = held_out(a, s, x, y, z, o[s]);
        if (M::f32_out(s)) {
            gstore_ptr<float>(a.out[s])[idx] = v;
        } else {
            const float w[1] = {v};
            store_field<S, 1>(a, s, x, y, z, w);
        }
    }
}

// ------------------------------------------------------ lane and tile helpers

// Lane l receives v from lane l-1 (l-1 >= 0) or `fill` (lane 0): DPP wave_shr:1.
__device__ __forceinline__ float lane_from_left(float v, float fill) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(fill), __float_as_int(v),
                                                      0x138, 0xF, 0xF, false));
}
// Lane l receives v from lane l+1 (l+1 <= 63) or `fill` (lane 63): DPP wave_shl:1.
__device__ __forceinline__ float lane_from_right(float v, float fill) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(fill), __float_as_int(v),
                                                      0x130, 0xF, 0xF, false));
}

__device__ __forceinline__ float bcast_lane(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous
// run of tiles (x fastest, then y, then z chunk) so that tiles sharing halo
// rows share that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int n) {
    constexpr int X = 8;
    const int q = n / X, r = n % X, xcd = b % X, i = b / X;
    return xcd < r ? xcd * (q + 1) + i : r * (q + 1) + (xcd - r) * q + i;
}

// ---- shared helpers of the tiled kernels --------------------------------

template <class M, class S, int VX>
__device__ __forceinline__ void load_raw(const StepArgs& a, int f, long long idx, float (&v)[VX]) {
    if (M::f32_field(f)) load_vec<StF32, VX>(a.in[f], idx, v);
    else load_vec<S, VX>(a.in[f], idx, v);
}

// Replace loaded values where a boundary rule fixes them: a ghost row or
// plane beyond a face, else held x faces, then a held row, then a held plane.
template <int VX>
__device__ __forceinline__ void fix_row(const StepArgs& a, int f, Src pz, Src py, int xl, float (&v)[VX]) {
    const bool ghost = py.cst == CST_GHOST || pz.cst == CST_GHOST;
    if (py.cst || pz.cst) {
        const float c = py.cst == CST_GHOST ? py.v : pz.cst == CST_GHOST ? pz.v : py.cst ? py.v : pz.v;
#pragma unroll
        for (int i = 0; i < VX; ++i) v[i] = c;
    }
    const int hm = a.held[f];
    if ((hm & 3) && !ghost) {
        const float b0 = a.bcv[f][0], b1 = a.bcv[f][1];
#pragma unroll
        for (int i = 0; i < VX; ++i) {
            const int x = xl + i;
            v[i] = ((hm & 1) && x == 0) ? b0 : ((hm & 2) && x == a.nx - 1) ? b1 : v[i];
        }
    }
}

// Value of row element `x` (0 <= x < nx <= TX) held by this wave: lane x/VX,
// element x%VX.  Every element is read out of that lane first and the choice
// is made among those values, so the window never needs an address.
template <int VX>
__device__ __forceinline__ float row_element(const float (&v)[VX], int x) {
    const int src = x / VX, e = x % VX;
    float t = bcast_lane(v[0], src);
#pragma unroll
    for (int i = 1; i < VX; ++i) {
        const float u = bcast_lane(v[i], src);
        t = e == i ? u : t;
    }
    return t;
}

// ---- plane-block kernel ---------------------------------------------------
//
// A workgroup computes the slab of columns [x0, x0+TX), rows [yb, yb+BY) and
// CZ planes [z0, z0+CZ).  All CZ+2 planes it reads (one halo plane on each
// side) are requested up front; the boundary rules of rows and planes are
// resolved once per slab.  There is no loop-carried window, so the compiler
// keeps every plane in fixed registers and lets all loads fly together.

// Rows exchanged between the waves of a workgroup, by plane parity: with two
// waves each exports the one row the other needs (wave 0 its last, wave 1
// its first); with more, every wave exports its first and last rows.
template <class M, int W, int TX>
struct BlockLds {
    static constexpr int EXP = W == 2 ? 1 : 2;
    float row[W > 1 ? 2 : 1][M::NF][W > 1 ? W : 1][EXP][W > 1 ? TX : 1];
};

// Lane l receives v from lane l-1, lane 0 from lane 63: DPP wave_ror:1.
__device__ __forceinline__ float lane_from_left_wrap(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x13C, 0xF, 0xF,
                                                      false));
}
// Lane l receives v from lane l+1, lane 63 from lane 0: DPP wave_rol:1.
__device__ __forceinline__ float lane_from_right_wrap(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x134, 0xF, 0xF,
                                                      false));
}

// Where the x neighbour outside a lane row comes from, per side of a tile:
// the loaded edge value (interior side or a wrapped/mirrored edge column),
// the cell's own value (mirror face), a fixed ghost value, or the lane
// rotation of a whole periodic row.
enum { XS_EDGE = 0, XS_OWN = 1, XS_CONST = 2, XS_ROT = 3 };

// x sides of a tile per field; returns whether any x-edge value must be
// loaded.  FAST (whole tiles, no fixed rows): interior sides and split
// periodic rows take the loaded edge, faces their rule.  Otherwise the
// ghosts come from lane reads (whole rows) or the loaded edges.
template <class M, bool FAST>
__device__ __forceinline__ bool x_sides(const StepArgs& a, int x0, int tx, bool whole_row, int (&xsl)[M::NF],
                                        int (&xsr)[M::NF]) {
    bool need_edges = false;
#pragma unroll
    for (int f = 0; f < M::NF; ++f) {
        const int klo = a.bck[f][0], khi = a.bck[f][1];
        const bool left_face = x0 == 0, right_face = x0 + tx >= a.nx;
        if (!FAST || whole_row) {
            xsl[f] = klo == BC_MIRROR ? XS_OWN : klo == BC_PERIODIC ? XS_ROT : XS_CONST;
            xsr[f] = khi == BC_MIRROR ? XS_OWN : khi == BC_PERIODIC ? XS_ROT : XS_CONST;
        }
        if (!whole_row) {
            xsl[f] = !left_face ? XS_EDGE : klo == BC_MIRROR ? XS_OWN : klo == BC_PERIODIC ? XS_EDGE : XS_CONST;
            xsr[f] = !right_face ? XS_EDGE : khi == BC_MIRROR ? XS_OWN : khi == BC_PERIODIC ? XS_EDGE : XS_CONST;
        }
        need_edges = need_edges || xsl[f] == XS_EDGE || xsr[f] == XS_EDGE;
    }
    return FAST ? need_edges : !whole_row;
}

// The cells of plane z that one wave owns.  v0 holds its RY rows of the
// plane, vm / vp the same rows of planes z-1 / z+1, h its halo rows (one
// wave: above and below; several: above for wave 0, below for the last),
// e the x-edge values (lane 0 left, lane 63 right).  Rows of neighbouring
// waves pass through LDS buffer `par`.  FAST takes the x ghosts from the
// side modes with no lane reads; otherwise from lane reads, with the ragged
// end of the row handled.  `held` applies held output faces.
template <class M, class S, int VX, int RY, int W, bool FAST>
__device__ __forceinline__ void plane_cells(const StepArgs& a, BlockLds<M, W, 64 * VX>& sm, int par, int lane,
                                            int w, int xl, int y0, int z, bool whole_row, bool held,
                                            const int (&xsl)[M::NF], const int (&xsr)[M::NF],
                                            const float (&vm)[M::NF][RY][VX], const float (&v0)[M::NF][RY][VX],
                                            const float (&vp)[M::NF][RY][VX],
                                            const float (&h)[M::NF][W == 1 ? 2 : 1][VX],
                                            const float (&e)[M::NF][RY]) {
    constexpr int NF = M::NF, NO = M::NO, TX = 64 * VX;
    constexpr int NH = W == 1 ? 2 : 1;
    float up[NF][VX], dn[NF][VX];
    if (W > 1) {
        constexpr int EXP = BlockLds<M, W, TX>::EXP;
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int i = 0; i < VX; ++i) {
                if (EXP == 1) {
                    sm.row[par][f][w][0][lane * VX + i] = w == 0 ? v0[f][RY - 1][i] : v0[f][0][i];
                } else {
                    sm.row[par][f][w][0][lane * VX + i] = v0[f][0][i];
                    sm.row[par][f][w][EXP - 1][lane * VX + i] = v0[f][RY - 1][i];
                }
            }
        __syncthreads();
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int i = 0; i < VX; ++i) {
                up[f][i] = w > 0 ? sm.row[par][f][w > 0 ? w - 1 : 0][EXP - 1][lane * VX + i] : h[f][0][i];
                dn[f][i] = w < W - 1 ? sm.row[par][f][w < W - 1 ? w + 1 : 0][0][lane * VX + i] : h[f][0][i];
            }
    } else {
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int i = 0; i < VX; ++i) {
                up[f][i] = h[f][0][i];
                dn[f][i] = h[f][NH - 1][i];
            }
    }
    const float uh = plane_wind<M>(a, z);
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int y = y0 + r;
        Nb n[NF][VX];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const float (&v)[VX] = v0[f][r];
            float left, right, R = 0.f;
            if (FAST) {
                // fill value of lane 0 (left) / lane 63 (right): no lane reads
                if (xsl[f] == XS_ROT) {
                    left = lane_from_left_wrap(v[VX - 1]);
                } else {
                    const float fl = xsl[f] == XS_OWN ? v[0] : xsl[f] == XS_CONST ? a.bcv[f][0] : e[f][r];
                    left = lane_from_left(v[VX - 1], fl);
                }
                if (xsr[f] == XS_ROT) {
                    right = lane_from_right_wrap(v[0]);
                } else {
                    const float fr = xsr[f] == XS_OWN ? v[VX - 1] : xsr[f] == XS_CONST ? a.bcv[f][1] : e[f][r];
                    right = lane_from_right(v[0], fr);
                }
            } else {
                float L;
                if (whole_row) {
                    const int klo = a.bck[f][0], khi = a.bck[f][1];
                    const float first = bcast_lane(v[0], 0);
                    const float last = row_element<VX>(v, a.nx - 1);
                    L = klo == BC_MIRROR ? first : klo == BC_PERIODIC ? last : a.bcv[f][0];
                    R = khi == BC_MIRROR ? last : khi == BC_PERIODIC ? first : a.bcv[f][1];
                } else {
                    L = bcast_lane(e[f][r], 0);
                    R = bcast_lane(e[f][r], 63);
                }
                left = lane_from_left(v[VX - 1], L);
                right = lane_from_right(v[0], R);
            }
#pragma unroll
            for (int i = 0; i < VX; ++i) {
                Nb& q = n[f][i];
                q.c = v[i];
                q.xm = i > 0 ? v[i - 1] : left;
                q.xp = i < VX - 1 ? v[i + 1] : right;
                if (!FAST && xl + i == a.nx - 1) q.xp = R;
                q.ym = r > 0 ? v0[f][r - 1][i] : up[f][i];
                q.yp = r < RY - 1 ? v0[f][r + 1][i] : dn[f][i];
                q.zm = vm[f][r][i];
                q.zp = vp[f][r][i];
            }
        }
        int s0 = 0, s1 = 0;
        if (M::SOURCES && y < a.ny) {
            s0 = cload_ptr<int>(a.src_row)[z * a.ny + y];
            s1 = cload_ptr<int>(a.src_row)[z * a.ny + y + 1];
        }
        float o[NO][VX];
#pragma unroll
        for (int i = 0; i < VX; ++i) {
            Nb ni[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) ni[f] = n[f][i];
            Emission<NO> em{};
            if (M::SOURCES && s0 < s1) em = cell_sources<NO>(a, xl + i, s0, s1);
            float oi[NO];
            M::cell(a, ni, uh, em.any, em.e, oi);
#pragma unroll
            for (int s = 0; s < NO; ++s) o[s][i] = held ? held_out(a, s, xl + i, y, z, oi[s]) : oi[s];
        }
        if (y < a.ny && xl < a.nx) {
            const long long idx = (long long)z * a.plane + (long long)y * a.pitch + xl;
#pragma unroll
            for (int s = 0; s < NO; ++s) {
                if (M::f32_out(s)) store_vec<StF32, VX>(a.out[s], idx, o[s]);
                else store_field<S, VX>(a, s, xl, y, z, o[s]);
            }
        }
    }
}

// The slab body keeps its own copy of the per-plane cell code (the same
// arithmetic as plane_cells, field-major register arrays): the generated code
// of this form is measurably faster for the slab kernel.
template <class M, class S, int VX, int RY, int W, int CZ, bool FAST>
__device__ __forceinline__ void block_compute(const StepArgs& a, BlockLds<M, W, 64 * VX>& sm, int lane, int w,
                                              int x0, int yb, int y0, int z0, int xl, bool whole_row,
                                              const Src (&rs)[M::NF][RY], const Src (&rh)[M::NF][W == 1 ? 2 : 1],
                                              const Src (&ps)[M::NF][CZ + 2]) {
    constexpr int NF = M::NF, NO = M::NO, TX = 64 * VX, NP = CZ + 2;
    constexpr int NH = W == 1 ? 2 : 1;
    const bool edge_wave = W == 1 || w == 0 || w == W - 1;

    // x sides of this tile, per field
    int xsl[NF], xsr[NF];
    bool need_edges = false;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const int klo = a.bck[f][0], khi = a.bck[f][1];
        const bool left_face = x0 == 0, right_face = x0 + TX >= a.nx;
        if (!FAST || whole_row) {
            // general path (and whole rows): sides from the face rule
            xsl[f] = klo == BC_MIRROR ? XS_OWN : klo == BC_PERIODIC ? XS_ROT : XS_CONST;
            xsr[f] = khi == BC_MIRROR ? XS_OWN : khi == BC_PERIODIC ? XS_ROT : XS_CONST;
        }
        if (!whole_row) {
            xsl[f] = !left_face ? XS_EDGE : klo == BC_MIRROR ? XS_OWN : klo == BC_PERIODIC ? XS_EDGE : XS_CONST;
            xsr[f] = !right_face ? XS_EDGE : khi == BC_MIRROR ? XS_OWN : khi == BC_PERIODIC ? XS_EDGE : XS_CONST;
        }
        need_edges = need_edges || xsl[f] == XS_EDGE || xsr[f] == XS_EDGE;
    }

    // issue every load of the slab
    float V[NF][NP][RY][VX];
    float H[NF][CZ][NH][VX];
    float E[NF][CZ][RY];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int k = 0; k < NP; ++k)
#pragma unroll
            for (int r = 0; r < RY; ++r)
                load_raw<M, S, VX>(a, f, (long long)ps[f][k].idx * a.plane +
                                             (long long)rs[f][r].idx * a.pitch + xl, V[f][k][r]);
    if (edge_wave) {
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int k = 0; k < CZ; ++k)
#pragma unroll
                for (int h = 0; h < NH; ++h)
                    load_raw<M, S, VX>(a, f, (long long)ps[f][k + 1].idx * a.plane +
                                                 (long long)rh[f][h].idx * a.pitch + xl, H[f][k][h]);
    }
    if (!FAST ? !whole_row : need_edges) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const int q = lane == 0 ? x0 - 1 : min(x0 + TX, a.nx);
            const int sxi = resolve_axis(q, a.nx, a.bck[f][0], a.bck[f][1], a.bcv[f][0], a.bcv[f][1]).idx;
#pragma unroll
            for (int k = 0; k < CZ; ++k)
#pragma unroll
                for (int r = 0; r < RY; ++r) {
                    E[f][k][r] = 0.f;
                    if (lane == 0 || lane == 63) {
                        const long long idx = (long long)ps[f][k + 1].idx * a.plane +
                                              (long long)rs[f][r].idx * a.pitch + sxi;
                        E[f][k][r] = M::f32_field(f) ? load1<StF32>(a.in[f], idx) : load1<S>(a.in[f], idx);
                    }
                }
        }
    }

    if (!FAST) {
        // boundary rules that replace loaded values (fixed rows/planes, held x faces)
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            bool any = (a.held[f] & 3) != 0;
#pragma unroll
            for (int k = 0; k < NP; ++k) any = any || ps[f][k].cst;
#pragma unroll
            for (int r = 0; r < RY; ++r) any = any || rs[f][r].cst;
#pragma unroll
            for (int h = 0; h < NH; ++h) any = any || rh[f][h].cst;
            if (any) {
#pragma unroll
                for (int k = 0; k < NP; ++k)
#pragma unroll
                    for (int r = 0; r < RY; ++r) fix_row<VX>(a, f, ps[f][k], rs[f][r], xl, V[f][k][r]);
                if (edge_wave) {
#pragma unroll
                    for (int k = 0; k < CZ; ++k)
#pragma unroll
                        for (int h = 0; h < NH; ++h) fix_row<VX>(a, f, ps[f][k + 1], rh[f][h], xl, H[f][k][h]);
                }
            }
            if (!whole_row) {
                const int q = lane == 0 ? x0 - 1 : min(x0 + TX, a.nx);
                const Src sx = resolve_axis(q, a.nx, a.bck[f][0], a.bck[f][1], a.bcv[f][0], a.bcv[f][1]);
#pragma unroll
                for (int k = 0; k < CZ; ++k)
#pragma unroll
                    for (int r = 0; r < RY; ++r) {
                        E[f][k][r] = fixed_or(sx, rs[f][r], ps[f][k + 1], E[f][k][r]);
                    }
            }
        }
    }

#pragma unroll
    for (int k = 1; k <= CZ; ++k) {
        const int z = z0 + k - 1;
        if (z < a.nz) {
            float up[NF][VX], dn[NF][VX];
            if (W > 1) {
                const int par = k & 1;
                constexpr int EXP = BlockLds<M, W, TX>::EXP;
#pragma unroll
                for (int f = 0; f < NF; ++f)
#pragma unroll
                    for (int i = 0; i < VX; ++i) {
                        if (EXP == 1) {
                            sm.row[par][f][w][0][lane * VX + i] = w == 0 ? V[f][k][RY - 1][i] : V[f][k][0][i];
                        } else {
                            sm.row[par][f][w][0][lane * VX + i] = V[f][k][0][i];
                            sm.row[par][f][w][EXP - 1][lane * VX + i] = V[f][k][RY - 1][i];
                        }
                    }
                __syncthreads();
#pragma unroll
                for (int f = 0; f < NF; ++f)
#pragma unroll
                    for (int i = 0; i < VX; ++i) {
                        up[f][i] = w > 0 ? sm.row[par][f][w > 0 ? w - 1 : 0][EXP - 1][lane * VX + i]
                                         : H[f][k - 1][0][i];
                        dn[f][i] = w < W - 1 ? sm.row[par][f][w < W - 1 ? w + 1 : 0][0][lane * VX + i]
                                             : H[f][k - 1][0][i];
                    }
            } else {
#pragma unroll
                for (int f = 0; f < NF; ++f)
#pragma unroll
                    for (int i = 0; i < VX; ++i) {
                        up[f][i] = H[f][k - 1][0][i];
                        dn[f][i] = H[f][k - 1][NH - 1][i];
                    }
            }
            const float uh = plane_wind<M>(a, z);
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                const int y = y0 + r;
                Nb n[NF][VX];
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const float (&v)[VX] = V[f][k][r];
                    float left, right, R = 0.f;
                    if (FAST) {
                        // fill value of lane 0 (left) / lane 63 (right): no lane reads
                        if (xsl[f] == XS_ROT) {
                            left = lane_from_left_wrap(v[VX - 1]);
                        } else {
                            const float fl = xsl[f] == XS_OWN ? v[0] : xsl[f] == XS_CONST ? a.bcv[f][0]
                                                                                          : E[f][k - 1][r];
                            left = lane_from_left(v[VX - 1], fl);
                        }
                        if (xsr[f] == XS_ROT) {
                            right = lane_from_right_wrap(v[0]);
                        } else {
                            const float fr = xsr[f] == XS_OWN ? v[VX - 1] : xsr[f] == XS_CONST ? a.bcv[f][1]
                                                                                               : E[f][k - 1][r];
                            right = lane_from_right(v[0], fr);
                        }
                    } else {
                        float L;
                        if (whole_row) {
                            const int klo = a.bck[f][0], khi = a.bck[f][1];
                            const float first = bcast_lane(v[0], 0);
                            const float last = row_element<VX>(v, a.nx - 1);
                            L = klo == BC_MIRROR ? first : klo == BC_PERIODIC ? last : a.bcv[f][0];
                            R = khi == BC_MIRROR ? last : khi == BC_PERIODIC ? first : a.bcv[f][1];
                        } else {
                            L = bcast_lane(E[f][k - 1][r], 0);
                            R = bcast_lane(E[f][k - 1][r], 63);
                        }
                        left = lane_from_left(v[VX - 1], L);
                        right = lane_from_right(v[0], R);
                    }
#pragma unroll
                    for (int i = 0; i < VX; ++i) {
                        Nb& q = n[f][i];
                        q.c = v[i];
                        q.xm = i > 0 ? v[i - 1] : left;
                        q.xp = i < VX - 1 ? v[i + 1] : right;
                        if (!FAST && xl + i == a.nx - 1) q.xp = R;
                        q.ym = r > 0 ? V[f][k][r - 1][i] : up[f][i];
                        q.yp = r < RY - 1 ? V[f][k][r + 1][i] : dn[f][i];
                        q.zm = V[f][k - 1][r][i];
                        q.zp = V[f][k + 1][r][i];
                    }
                }
                int s0 = 0, s1 = 0;
                if (M::SOURCES && y < a.ny) {
                    s0 = a.src_row[z * a.ny + y];
                    s1 = a.src_row[z * a.ny + y + 1];
                }
                float o[NO][VX];
#pragma unroll
                for (int i = 0; i < VX; ++i) {
                    Nb ni[NF];
#pragma unroll
                    for (int f = 0; f < NF; ++f) ni[f] = n[f][i];
                    Emission<NO> em{};
                    if (M::SOURCES && s0 < s1) em = cell_sources<NO>(a, xl + i, s0, s1);
                    float oi[NO];
                    M::cell(a, ni, uh, em.any, em.e, oi);
#pragma unroll
                    for (int s = 0; s < NO; ++s) o[s][i] = FAST ? oi[s] : held_out(a, s, xl + i, y, z, oi[s]);
                }
                if (y < a.ny && xl < a.nx) {
                    const long long idx = (long long)z * a.plane + (long long)y * a.pitch + xl;
#pragma unroll
                    for (int s = 0; s < NO; ++s) {
                        if (M::f32_out(s)) store_vec<StF32, VX>(a.out[s], idx, o[s]);
                        else store_field<S, VX>(a, s, xl, y, z, o[s]);
                    }
                }
            }
        }
    }
}

template <class M, class S, int VX, int RY, int W, int CZ>
__device__ __forceinline__ void block_step(const StepArgs& a, int t, BlockLds<M, W, 64 * VX>& sm) {
    constexpr int NF = M::NF, NO = M::NO, TX = 64 * VX, BY = RY * W, NP = CZ + 2;
    constexpr int NH = W == 1 ? 2 : 1;      // halo rows a wave loads per plane
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const TileXYZ tc = tile_coords(a, t);
    const int x0 = tc.x * TX;
    const int yb = tc.y * BY;
    const int y0 = yb + w * RY;
    const int z0 = tc.z * CZ;
    const int xl = x0 + lane * VX;
    const bool whole_row = a.tiles_x == 1;
    // halo row h of this wave: W == 1: h=0 above, h=1 below; else above for
    // wave 0, below for wave W-1.
    const int hrow0 = (W == 1 || w == 0) ? yb - 1 : yb + BY;

    // z-independent row sources and z plane sources, resolved once per slab.
    // A slab two or more cells inside every y and z face reads only its own
    // rows and planes: no rule applies there.
    Src rs[NF][RY], rh[NF][NH], ps[NF][NP];
    bool fast = a.nx % TX == 0;
    const bool inside = yb >= 2 && yb + BY <= a.ny - 2 && z0 >= 2 && z0 + CZ <= a.nz - 2;
    if (inside) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
#pragma unroll
            for (int r = 0; r < RY; ++r) rs[f][r] = Src{y0 + r, 0, 0.f};
#pragma unroll
            for (int h = 0; h < NH; ++h) rh[f][h] = Src{h == 0 ? hrow0 : yb + BY, 0, 0.f};
#pragma unroll
            for (int k = 0; k < NP; ++k) ps[f][k] = Src{z0 - 1 + k, 0, 0.f};
            fast = fast && (a.held[f] & 3) == 0;
        }
    } else {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                rs[f][r] = resolve_axis(y0 + r, a.ny, a.bck[f][2], a.bck[f][3], a.bcv[f][2], a.bcv[f][3]);
                fast = fast && !rs[f][r].cst;
            }
#pragma unroll
            for (int h = 0; h < NH; ++h) {
                rh[f][h] = resolve_axis(h == 0 ? hrow0 : yb + BY, a.ny, a.bck[f][2], a.bck[f][3],
                                        a.bcv[f][2], a.bcv[f][3]);
                fast = fast && !rh[f][h].cst;
            }
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                ps[f][k] = resolve_axis(z0 - 1 + k, a.nz, a.bck[f][4], a.bck[f][5], a.bcv[f][4], a.bcv[f][5]);
                fast = fast && !ps[f][k].cst;
            }
            fast = fast && (a.held[f] & 3) == 0;
        }
    }
    // outputs on a held face of this slab need the held value
#pragma unroll
    for (int s = 0; s < NO; ++s) {
        const int hm = a.out_held[s];
        const bool touches = ((hm & 1) && x0 == 0) || ((hm & 2) && x0 + TX >= a.nx) ||
                             ((hm & 4) && yb == 0) || ((hm & 8) && yb + BY >= a.ny) ||
                             ((hm & 16) && z0 == 0) || ((hm & 32) && z0 + CZ >= a.nz);
        fast = fast && !touches;
    }
    if (fast) block_compute<M, S, VX, RY, W, CZ, true>(a, sm, lane, w, x0, yb, y0, z0, xl, whole_row, rs, rh, ps);
    else block_compute<M, S, VX, RY, W, CZ, false>(a, sm, lane, w, x0, yb, y0, z0, xl, whole_row, rs, rh, ps);
    if (W > 1) __syncthreads();   // the LDS rows may be reused by the next slab
}

template <class M, class S, int VX, int RY, int W, int CZ>
__global__ __launch_bounds__(64 * W) void block_kernel(const StepArgs* __restrict__ pa) {
    __shared__ BlockLds<M, W, 64 * VX> sm;
    tick_clock<M>(*pa, (blockIdx.x | threadIdx.x) == 0);
    block_step<M, S, VX, RY, W, CZ>(*pa, xcd_tile(blockIdx.x, gridDim.x), sm);
}

// ---- z-march kernel -------------------------------------------------------
//
// A workgroup owns columns [x0, x0+TX) and rows [yb, yb+BY) and marches planes
// [z0, z1), reading each plane of its rows once.  Each wave keeps NB = 3+PF
// planes in a register ring: z-1, z, z+1 in use and PF more in flight.  The
// march is unrolled by NB so that every ring slot is a fixed set of registers
// (no moves).  Rows and x sides are resolved once per tile; a plane needs a
// fix-up only where a rule replaces loaded values (a fixed or held z face, or
// the tile's fixed rows and held x faces in the general path).

template <class M, class S, int VX, int RY, int W, int PF, bool FAST>
__device__ __forceinline__ void march_tile(const StepArgs& a, BlockLds<M, W, 64 * VX>& sm, int lane, int w,
                                           int x0, int y0, int z0, int z1, int xl, bool whole_row,
                                           const Src (&rs)[M::NF][RY], const Src (&rh)[M::NF][W == 1 ? 2 : 1],
                                           bool rows_fix, bool xy_held, bool held_lo, bool held_hi) {
    constexpr int NF = M::NF, TX = 64 * VX, NB = 3 + PF;
    constexpr int NH = W == 1 ? 2 : 1;
    const bool edge_wave = W == 1 || w == 0 || w == W - 1;
    int xsl[NF], xsr[NF];
    const bool need_edges = x_sides<M, FAST>(a, x0, TX, whole_row, xsl, xsr);
    const int q = lane == 0 ? x0 - 1 : min(x0 + TX, a.nx);
    int sxi[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f)
        sxi[f] = resolve_axis(q, a.nx, a.bck[f][0], a.bck[f][1], a.bcv[f][0], a.bcv[f][1]).idx;

    float V[NB][NF][RY][VX];
    float H[NB][NF][NH][VX];
    float E[NB][NF][RY];

    // request plane p (halo rows and x edges only for planes this tile computes)
    auto issue = [&](float (&v)[NF][RY][VX], float (&hv)[NF][NH][VX], float (&e)[NF][RY], int p) __attribute__((always_inline)) {
        const bool extras = p >= z0 && p < z1;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const int pz = resolve_axis(p, a.nz, a.bck[f][4], a.bck[f][5], a.bcv[f][4], a.bcv[f][5]).idx;
            const long long pb = (long long)pz * a.plane;
#pragma unroll
            for (int r = 0; r < RY; ++r)
                load_raw<M, S, VX>(a, f, pb + (long long)rs[f][r].idx * a.pitch + xl, v[f][r]);
            if (extras && edge_wave) {
#pragma unroll
                for (int k = 0; k < NH; ++k)
                    load_raw<M, S, VX>(a, f, pb + (long long)rh[f][k].idx * a.pitch + xl, hv[f][k]);
            }
            if (extras && need_edges) {
#pragma unroll
                for (int r = 0; r < RY; ++r) {
                    e[f][r] = 0.f;
                    if (lane == 0 || lane == 63) {
                        const long long idx = pb + (long long)rs[f][r].idx * a.pitch + sxi[f];
                        e[f][r] = M::f32_field(f) ? load1<StF32>(a.in[f], idx) : load1<S>(a.in[f], idx);
                    }
                }
            }
        }
    };
    // replace loaded values of plane p where a boundary rule fixes them
    auto finish = [&](float (&v)[NF][RY][VX], float (&hv)[NF][NH][VX], float (&e)[NF][RY], int p) __attribute__((always_inline)) {
        bool any = rows_fix;
        if (p <= 0 || p >= a.nz - 1) {
#pragma unroll
            for (int f = 0; f < NF; ++f)
                any = any || resolve_axis(p, a.nz, a.bck[f][4], a.bck[f][5], a.bcv[f][4], a.bcv[f][5]).cst;
        }
        if (any) {
            const bool extras = p >= z0 && p < z1;
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const Src pz = resolve_axis(p, a.nz, a.bck[f][4], a.bck[f][5], a.bcv[f][4], a.bcv[f][5]);
#pragma unroll
                for (int r = 0; r < RY; ++r) fix_row<VX>(a, f, pz, rs[f][r], xl, v[f][r]);
                if (extras && edge_wave) {
#pragma unroll
                    for (int k = 0; k < NH; ++k) fix_row<VX>(a, f, pz, rh[f][k], xl, hv[f][k]);
                }
                if (extras && need_edges) {
                    const Src sx = resolve_axis(q, a.nx, a.bck[f][0], a.bck[f][1], a.bcv[f][0], a.bcv[f][1]);
#pragma unroll
                    for (int r = 0; r < RY; ++r) e[f][r] = fixed_or(sx, rs[f][r], pz, e[f][r]);
                }
            }
        }
    };

    // planes z0-1 .. z0+1+PF go to slots 0 .. NB-1; plane p lives in slot (p - z0 + 1) % NB
#pragma unroll
    for (int k = 0; k < NB; ++k)
        if (z0 - 1 + k <= z1) issue(V[k], H[k], E[k], z0 - 1 + k);
#pragma unroll
    for (int k = 0; k < 3; ++k) finish(V[k], H[k], E[k], z0 - 1 + k);

    for (int zb = z0; zb < z1; zb += NB) {
#pragma unroll
        for (int J = 0; J < NB; ++J) {
            const int z = zb + J;
            if (z < z1) {
                const bool held = xy_held || (held_lo && z == 0) || (held_hi && z == a.nz - 1);
                plane_cells<M, S, VX, RY, W, FAST>(a, sm, (z - z0) & 1, lane, w, xl, y0, z, whole_row, held,
                                                   xsl, xsr, V[J], V[(J + 1) % NB], V[(J + 2) % NB],
                                                   H[(J + 1) % NB], E[(J + 1) % NB]);
                // the slot of plane z-1 is free: request plane z+2+PF into it
                if (z + 2 + PF <= z1) issue(V[J], H[J], E[J], z + 2 + PF);
                if (z + 2 <= z1) finish(V[(J + 3) % NB], H[(J + 3) % NB], E[(J + 3) % NB], z + 2);
            }
        }
    }
}

template <class M, class S, int VX, int RY, int W, int PF>
__device__ __forceinline__ void tile_step(const StepArgs& a, int t, BlockLds<M, W, 64 * VX>& sm) {
    constexpr int NF = M::NF, NO = M::NO, TX = 64 * VX, BY = RY * W;
    constexpr int NH = W == 1 ? 2 : 1;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const TileXYZ tc = tile_coords(a, t);
    const int x0 = tc.x * TX;
    const int yb = tc.y * BY;
    const int y0 = yb + w * RY;
    const int z0 = tc.z * a.cz;
    const int z1 = min(z0 + a.cz, a.nz);
    const int xl = x0 + lane * VX;
    const bool whole_row = a.tiles_x == 1;
    const int hrow0 = (W == 1 || w == 0) ? yb - 1 : yb + BY;

    // rows of this wave and its halo rows, resolved once for the whole march
    Src rs[NF][RY], rh[NF][NH];
    bool rows_fix = false;
    const int ql = x0 - 1, qr = min(x0 + TX, a.nx);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            rs[f][r] = resolve_axis(y0 + r, a.ny, a.bck[f][2], a.bck[f][3], a.bcv[f][2], a.bcv[f][3]);
            rows_fix = rows_fix || rs[f][r].cst;
        }
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            rh[f][h] = resolve_axis(h == 0 ? hrow0 : yb + BY, a.ny, a.bck[f][2], a.bck[f][3], a.bcv[f][2],
                                    a.bcv[f][3]);
            rows_fix = rows_fix || rh[f][h].cst;
        }
        rows_fix = rows_fix || (a.held[f] & 3) != 0;
        if (!whole_row)
            rows_fix = rows_fix ||
                       resolve_axis(ql, a.nx, a.bck[f][0], a.bck[f][1], a.bcv[f][0], a.bcv[f][1]).cst ||
                       resolve_axis(qr, a.nx, a.bck[f][0], a.bck[f][1], a.bcv[f][0], a.bcv[f][1]).cst;
    }
    // held output faces: x and y faces this tile touches hold on every plane
    bool xy_held = false, held_lo = false, held_hi = false;
#pragma unroll
    for (int s = 0; s < NO; ++s) {
        const int hm = a.out_held[s];
        xy_held = xy_held || ((hm & 1) && x0 == 0) || ((hm & 2) && x0 + TX >= a.nx) || ((hm & 4) && yb == 0) ||
                  ((hm & 8) && yb + BY >= a.ny);
        held_lo = held_lo || (hm & 16);
        held_hi = held_hi || (hm & 32);
    }
    const bool fast = a.nx % TX == 0 && !rows_fix;
    if (fast)
        march_tile<M, S, VX, RY, W, PF, true>(a, sm, lane, w, x0, y0, z0, z1, xl, whole_row, rs, rh, false,
                                              xy_held, held_lo, held_hi);
    else
        march_tile<M, S, VX, RY, W, PF, false>(a, sm, lane, w, x0, y0, z0, z1, xl, whole_row, rs, rh, rows_fix,
                                               xy_held, held_lo, held_hi);
    if (W > 1) __syncthreads();   // the LDS rows may be reused by the next tile
}

// Step arguments live in device memory (not the kernel-argument segment) so
// that boundary values picked by runtime conditions are plain scalar loads.
template <class M, class S, int VX, int RY, int W, int PF>
__global__ __launch_bounds__(64 * W) void tiled_kernel(const StepArgs* __restrict__ pa) {
    __shared__ BlockLds<M, W, 64 * VX> sm;
    tick_clock<M>(*pa, (blockIdx.x | threadIdx.x) == 0);
    tile_step<M, S, VX, RY, W, PF>(*pa, xcd_tile(blockIdx.x, gridDim.x), sm);
}

// ---- LDS-ring z-march kernel ------------------------------------------------
//
// Whole rows of 256*(NCH-1) < nx <= 256*NCH FP32 cells (nx a multiple of 4;
// the lanes past the row end in the last 256-cell chunk load, compute and
// store nothing of use).  A workgroup owns rows [yb, yb+BY)
// and marches planes [z0, z1).  One producer wave streams every plane it
// needs (its BY rows plus one halo row on each side, every field) from HBM
// into a ring of D plane slots in LDS with global_load_lds_dwordx4, so the
// data in flight holds no registers; WC consumer waves compute from the ring.
// The producer issues nothing but these loads, so it can wait for one plane
// with an exact vmcnt, and one barrier per plane hands the plane over.  While
// plane z is computed, planes z-1, z, z+1 are in use and D-3 more are in
// flight.  The consumers' LDS reads and the producer's loads sit in separate
// loops, so the compiler never drains the loads for an LDS read.

template <int K>
__device__ __forceinline__ void vm_wait_imm() {
    static_assert(K >= 0 && K <= 63, "vmcnt holds 6 bits");
    // s_waitcnt fields: vmcnt [3:0] and [15:14], expcnt [6:4], lgkmcnt [11:8]
    __builtin_amdgcn_s_waitcnt((K & 15) | (((K >> 4) & 3) << 14) | (7 << 4) | (15 << 8));
}

// vmcnt(n * STEP) for a run-time n in [0, N]
template <int STEP, int N>
__device__ __forceinline__ void vm_wait_steps(int n) {
    if (n >= N) {
        vm_wait_imm<N * STEP>();
    } else if constexpr (N > 0) {
        vm_wait_steps<STEP, N - 1>(n);
    }
}

// A workgroup barrier the compiler may not move memory accesses across, with
// no fence: a fence would wait for every load in flight.
// s_waitcnt vmcnt(n) for a run-time n in [LO, HI] (a tree of immediates)
template <int LO, int HI>
__device__ __forceinline__ void vm_wait_count(int n) {
    if constexpr (LO == HI) {
        vm_wait_imm<LO>();
    } else {
        constexpr int MID = (LO + HI) / 2;
        if (n <= MID) vm_wait_count<LO, MID>(n);
        else vm_wait_count<MID + 1, HI>(n);
    }
}

__device__ __forceinline__ void ring_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Ring of D plane slots of NF fields x (BY+2) rows x 256*NCH cells of ES
// bytes.  A lane loads 16 bytes (16/ES cells) per instruction, so a row takes
// NQ loads: NCH for FP32, half as many for 2-byte cells.
template <int NF, int NCH, int BY, int D, int ES = 4>
struct LdsRing {
    static constexpr int ROWS = BY + 2, TXT = 256 * NCH, SLOT = NF * ROWS * TXT;   // cells
    static constexpr int CPL = 16 / ES, CPQ = 64 * CPL;        // cells per lane / per load
    static constexpr int NQ = (TXT + CPQ - 1) / CPQ;           // loads per row
    static constexpr int CH = NF * ROWS * NQ;                  // loads per plane
    static constexpr int SLOT_W = SLOT * ES / 4;               // a slot in 4-byte words
    static constexpr long long BYTES = (long long)ES * D * SLOT;
    static constexpr bool FITS = BYTES <= 160 * 1024 && (D - 4) * CH <= 63 && D >= 4;
};

// (The body is compiled for the device only: the host compiler fails to
// reuse this specialization once a kernel of each stencil form asked for it.)
template <class M, class S, int NCH, int BY, int WC, int D>
__device__ __forceinline__ void lds_producer(const StepArgs& a, RD_LDS float* ring, int yb, int z0, int z1) {
#ifndef __HIP_DEVICE_COMPILE__
    (void)a, (void)ring, (void)yb, (void)z0, (void)z1;
#else
    using T = typename S::T;
    using R = LdsRing<M::NF, NCH, BY, D, int(sizeof(T))>;
    constexpr int NF = M::NF, ROWS = R::ROWS, TXT = R::TXT, CPL = R::CPL, CPQ = R::CPQ, NQ = R::NQ;
    const int lane = threadIdx.x & 63;
    const bool in_row = lane * CPL < a.nx - CPQ * (NQ - 1);      // of a row's last load
    // grid row of LDS row j is yb - 1 + j, resolved by the face rules
    int ridx[NF][ROWS];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int j = 0; j < ROWS; ++j)
            ridx[f][j] = resolve_axis(yb - 1 + j, a.ny, a.bck[f][2], a.bck[f][3], a.bcv[f][2], a.bcv[f][3]).idx;
    auto issue = [&](RD_LDS float* slot, int p) __attribute__((always_inline)) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const int pz = resolve_axis(p, a.nz, a.bck[f][4], a.bck[f][5], a.bcv[f][4], a.bcv[f][5]).idx;
            const RD_GLOBAL T* base = gload_ptr<T>(a.in[f]) + (long long)pz * a.plane + lane * CPL;
            RD_LDS T* slot_t = (RD_LDS T*)slot;
#pragma unroll
            for (int j = 0; j < ROWS; ++j)
#pragma unroll
                for (int q = 0; q < NQ; ++q)
                    if (q < NQ - 1 || in_row)
                        __builtin_amdgcn_global_load_lds(base + (long long)ridx[f][j] * a.pitch + q * CPQ,
                                                         (RD_LDS void*)(slot_t + (f * ROWS + j) * TXT + q * CPQ), 16, 0,
                                                         0);
        }
    };
    // planes z0-1 .. z0+D-3 into slots 0 .. D-2; plane p lives in slot (p - z0 + 1) % D
#pragma unroll
    for (int k = 0; k < D - 1; ++k)
        if (z0 - 1 + k <= z1) issue(ring + k * R::SLOT_W, z0 - 1 + k);
    for (int zb = z0; zb < z1; zb += D) {
#pragma unroll
        for (int J = 0; J < D; ++J) {
            const int z = zb + J;
            if (z < z1) {
                // plane z+1 complete: the loads issued after it are planes z+2 ..
                vm_wait_steps<R::CH, D - 4>(min(D - 4, z1 - z - 1));
                ring_barrier();
                // every consumer is past plane z-1, so the slot of plane z-2 is free
                if (z + D - 2 <= z1) issue(ring + ((J + D - 1) % D) * R::SLOT_W, z + D - 2);
            }
        }
    }
#endif
}

template <class M, class ST, int NCH, int BY, int WC, int D, bool S19>
__device__ __forceinline__ void lds_consumer(const StepArgs& a, const RD_LDS float* ring_w, int cw, int yb, int z0,
                                             int z1) {
    using T = typename ST::T;
    using R = LdsRing<M::NF, NCH, BY, D, int(sizeof(T))>;
    const RD_LDS T* ring = (const RD_LDS T*)ring_w;     // cells of the storage type
    constexpr int NF = M::NF, NO = M::NO, TXT = R::TXT, RY = BY / WC;
    using NBT = std::conditional_t<S19, Nb19, Nb>;
    const int lane = threadIdx.x & 63;
    const int r0 = cw * RY;                   // first tile row of this wave
    // rows r0-1 .. r0+RY of the tile (LDS rows r0 .. r0+RY+1), for fix-ups
    Src rs[NF][RY + 2];
    bool rows_fix = false;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
#pragma unroll
        for (int r = 0; r < RY + 2; ++r) {
            rs[f][r] = resolve_axis(yb + r0 - 1 + r, a.ny, a.bck[f][2], a.bck[f][3], a.bcv[f][2], a.bcv[f][3]);
            rows_fix = rows_fix || rs[f][r].cst;
        }
        rows_fix = rows_fix || (a.held[f] & 3) != 0;
    }
    // the last cell of a row sits in lane `last` of the last chunk
    const int last = ((a.nx - 256 * (NCH - 1)) >> 2) - 1;
    const bool at_end = lane == last;
    // x sides of a whole row: rotate (periodic), own edge value (mirror) or
    // the face value, held in registers across the plane loop
    int xsl[NF], xsr[NF];
    (void)x_sides<M, true>(a, 0, TXT, true, xsl, xsr);
    bool rot_l[NF], own_l[NF], rot_r[NF], own_r[NF];
    float fill_l[NF], fill_r[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        rot_l[f] = xsl[f] == XS_ROT;
        own_l[f] = xsl[f] == XS_OWN;
        rot_r[f] = xsr[f] == XS_ROT;
        own_r[f] = xsr[f] == XS_OWN;
        fill_l[f] = a.bcv[f][0];
        fill_r[f] = a.bcv[f][1];
    }
    bool xy_held = false, held_lo = false, held_hi = false;
#pragma unroll
    for (int s = 0; s < NO; ++s) {
        const int hm = a.out_held[s];
        xy_held = xy_held || (hm & 3) || ((hm & 4) && yb + r0 == 0) || ((hm & 8) && yb + r0 + RY >= a.ny);
        held_lo = held_lo || (hm & 16);
        held_hi = held_hi || (hm & 32);
    }

    // Rows r0-1 .. r0+RY of planes z-1, z, z+1 (LDS rows r0 .. r0+RY+1), with
    // the face rules applied.  Plane z of one step is plane z-1 of the next,
    // with the same rules, so each step reads plane z+1 alone from the ring;
    // the plane loop is unrolled three times so that the three register
    // planes trade roles without copies.  The first plane z0-1 needs only the
    // wave's own rows for the 7-point form (halo = false).
    using Plane = float[NF][RY + 2][NCH][4];
    Plane PA, PB, PC;
    // four cells of a lane: one 16-byte LDS read (FP32) or one 8-byte read
    // unpacked to FP32 (2-byte storage)
    auto ld4 = [&](const RD_LDS T* q, float (&o)[4]) __attribute__((always_inline)) {
        if constexpr (sizeof(T) == 4) {
            lds_ld4((const RD_LDS float*)q, o);
        } else {
            typedef unsigned lds_v2 __attribute__((ext_vector_type(2)));
            const lds_v2 t = *(const RD_LDS lds_v2*)q;
            o[0] = ST::up(T(t.x & 0xffffu));
            o[1] = ST::up(T(t.x >> 16));
            o[2] = ST::up(T(t.y & 0xffffu));
            o[3] = ST::up(T(t.y >> 16));
        }
    };
    auto load_plane = [&](const RD_LDS T* P, Plane& v, bool halo) __attribute__((always_inline)) {
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int c = 0; c < NCH; ++c)
#pragma unroll
                for (int r = 0; r < RY + 2; ++r)
                    if (halo || (r > 0 && r <= RY))
                        ld4(P + (f * R::ROWS + r0 + r) * TXT + c * 256 + lane * 4, v[f][r][c]);
    };
    // boundary rules that replace loaded values (fixed or held rows, the
    // planes at and beyond the z faces, x faces)
    auto fix_plane = [&](int p, Plane& v, bool halo) __attribute__((always_inline)) {
        if (rows_fix || p <= 0 || p >= a.nz - 1) {
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const Src ps = resolve_axis(p, a.nz, a.bck[f][4], a.bck[f][5], a.bcv[f][4], a.bcv[f][5]);
#pragma unroll
                for (int c = 0; c < NCH; ++c)
#pragma unroll
                    for (int r = 0; r < RY + 2; ++r)
                        if (halo || (r > 0 && r <= RY))
                            fix_row<4>(a, f, ps, rs[f][r], c * 256 + lane * 4, v[f][r][c]);
            }
        }
    };

    int sp_slot = 2;                 // slot of plane z+1 (plane z0-1 is slot 0)
    // one plane: vm, v0 hold planes z-1, z; plane z+1 is read into vp
    auto plane = [&](int z, Plane& vm, Plane& v0, Plane& vp, bool first) __attribute__((always_inline)) {
        {
            {
                // scalar loads of this plane's wind and source range go out
                // before the barrier so their latency hides behind it
                const float uh = plane_wind<M>(a, z);
                bool plane_src = false;
                if (M::SOURCES) {
                    const int pa0 = cload_ptr<int>(a.src_row)[z * a.ny];
                    const int pa1 = cload_ptr<int>(a.src_row)[(z + 1) * a.ny];
                    plane_src = pa0 < pa1;
                }
                ring_barrier();
                if (first) {
                    load_plane(ring, vm, S19);
                    load_plane(ring + R::SLOT, v0, true);
                    fix_plane(z - 1, vm, S19);
                    fix_plane(z, v0, true);
                }
                load_plane(ring + sp_slot * R::SLOT, vp, true);
                sp_slot = sp_slot + 1 == D ? 0 : sp_slot + 1;
                fix_plane(z + 1, vp, true);
                const bool held = xy_held || (held_lo && z == 0) || (held_hi && z == a.nz - 1);
#pragma unroll
                for (int r = 0; r < RY; ++r) {
                    const int y = yb + r0 + r;
                    NBT n[NF][NCH][4];
                    // x neighbours of a row across lanes, chunks and the x
                    // faces; `k` scales the face value (a cross sum of four)
                    auto xnb = [&](int f, const float (&row)[NCH][4], int c, float k, float& left, float& right)
                                   __attribute__((always_inline)) {
                        const float fl = c > 0 ? lane_from_left_wrap(row[c - 1][3])
                                         : rot_l[f] ? bcast_lane(row[NCH - 1][3], last)
                                         : own_l[f] ? row[0][0] : k * fill_l[f];
                        const float fr = c < NCH - 1 ? lane_from_right_wrap(row[c + 1][0])
                                         : rot_r[f] ? bcast_lane(row[0][0], 0)
                                         : own_r[f] ? row[NCH - 1][3] : k * fill_r[f];
                        left = lane_from_left(row[c][3], fl);
                        right = lane_from_right(row[c][0], fr);
                        if (c == NCH - 1) right = at_end ? fr : right;
                    };
#pragma unroll
                    for (int f = 0; f < NF; ++f) {
                        // 19 points: the cross sums of this row and their x neighbours
                        float sc[NCH][4];
                        if constexpr (S19) {
#pragma unroll
                            for (int c = 0; c < NCH; ++c)
#pragma unroll
                                for (int i = 0; i < 4; ++i)
                                    sc[c][i] = (v0[f][r][c][i] + v0[f][r + 2][c][i]) + (vm[f][r + 1][c][i] + vp[f][r + 1][c][i]);
                        }
#pragma unroll
                        for (int c = 0; c < NCH; ++c) {
                            const float (&v)[4] = v0[f][r + 1][c];
                            float left, right;
                            xnb(f, v0[f][r + 1], c, 1.f, left, right);
                            float sl = 0.f, sr = 0.f;
                            if constexpr (S19) xnb(f, sc, c, 4.f, sl, sr);
#pragma unroll
                            for (int i = 0; i < 4; ++i) {
                                NBT& q = n[f][c][i];
                                q.c = v[i];
                                q.xm = i > 0 ? v[i - 1] : left;
                                q.xp = i < 3 ? v[i + 1] : right;
                                q.ym = v0[f][r][c][i];
                                q.yp = v0[f][r + 2][c][i];
                                q.zm = vm[f][r + 1][c][i];
                                q.zp = vp[f][r + 1][c][i];
                                if constexpr (S19) {
                                    q.s = sc[c][i];
                                    q.sxm = i > 0 ? sc[c][i - 1] : sl;
                                    q.sxp = i < 3 ? sc[c][i + 1] : sr;
                                    q.q = (vm[f][r][c][i] + vm[f][r + 2][c][i]) + (vp[f][r][c][i] + vp[f][r + 2][c][i]);
                                }
                            }
                        }
                    }
                    int s0 = 0, s1 = 0;
                    if (M::SOURCES && plane_src && y < a.ny) {
                        s0 = cload_ptr<int>(a.src_row)[z * a.ny + y];
                        s1 = cload_ptr<int>(a.src_row)[z * a.ny + y + 1];
                    }
#pragma unroll
                    for (int c = 0; c < NCH; ++c) {
                        const int xl = c * 256 + lane * 4;
                        float o[NO][4];
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            NBT ni[NF];
#pragma unroll
                            for (int f = 0; f < NF; ++f) ni[f] = n[f][c][i];
                            Emission<NO> em{};
                            if (M::SOURCES && s0 < s1) em = cell_sources<NO>(a, xl + i, s0, s1);
                            float oi[NO];
                            M::cell(a, ni, uh, em.any, em.e, oi);
#pragma unroll
                            for (int s = 0; s < NO; ++s) o[s][i] = held ? held_out(a, s, xl + i, y, z, oi[s]) : oi[s];
                        }
                        if (y < a.ny && (c < NCH - 1 || lane <= last)) {
                            const long long idx = (long long)z * a.plane + (long long)y * a.pitch + xl;
#pragma unroll
                            for (int s = 0; s < NO; ++s) {
                                if (M::f32_out(s)) store_vec<StF32, 4>(a.out[s], idx, o[s]);
                                else store_field<ST, 4>(a, s, xl, y, z, o[s]);
                            }
                        }
                    }
                }
            }
        }
    };
    for (int z = z0; z < z1; z += 3) {
        plane(z, PA, PB, PC, z == z0);
        if (z + 1 >= z1) break;
        plane(z + 1, PB, PC, PA, false);
        if (z + 2 >= z1) break;
        plane(z + 2, PC, PA, PB, false);
    }
}

template <class M, class S, int NCH, int BY, int WC, int D, bool S19>
__global__ __launch_bounds__(64 * (WC + 1)) void lds_kernel(const StepArgs* __restrict__ pa) {
    using R = LdsRing<M::NF, NCH, BY, D, int(sizeof(typename S::T))>;
    static_assert(R::FITS && BY % WC == 0, "ring shape does not fit");
    __shared__ __attribute__((aligned(16))) float ring[D * R::SLOT_W];
    const StepArgs& a = *pa;
    tick_clock<M>(a, (blockIdx.x | threadIdx.x) == 0);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const TileXYZ tc = tile_coords(a, xcd_tile(blockIdx.x, gridDim.x));
    const int yb = tc.y * BY;
    const int z0 = tc.z * a.cz;
    const int z1 = min(z0 + a.cz, a.nz);
    RD_LDS float* base = (RD_LDS float*)&ring[0];
    if (w == 0) lds_producer<M, S, NCH, BY, WC, D>(a, base, yb, z0, z1);
    else lds_consumer<M, S, NCH, BY, WC, D, S19>(a, base, w - 1, yb, z0, z1);
}

// ---- two steps per launch (temporal blocking) on the LDS ring ---------------
//
// The same producer / consumer split, two time levels per pass over HBM: the
// input ring holds planes of rows yb-2 .. yb+BY+1 (a halo of two), and the
// consumers first compute the intermediate level ("mid") on rows yb-1 ..
// yb+BY into a ring of four LDS planes, then the output level on rows yb ..
// yb+BY-1 from the mid ring.  Iteration q computes mid plane q and output
// plane q-2, so one barrier per plane covers both rings.  A mid value the
// output needs from outside the grid follows the face rule: periodic ones
// are computed from wrapped inputs, mirror ones are the edge row or plane,
// fixed ones the face value.  Every cell goes through the same cell function
// as a single step, so two steps here give the bits of two single steps.
// Models with point sources are not blocked.

template <int NF, int NCH, int BY, int D>
struct Lds2Ring {
    static constexpr int IROWS = BY + 4, MROWS = BY + 2, TXT = 256 * NCH;
    static constexpr int ISLOT = NF * IROWS * TXT, MSLOT = NF * MROWS * TXT;
    static constexpr int CH = NF * IROWS * NCH;                // 1 KB loads per input plane
    static constexpr long long BYTES = 4LL * (D * ISLOT + 4 * MSLOT);
    static constexpr bool FITS = BYTES <= 160 * 1024 && (D - 4) * CH <= 63 && D >= 4;
};

// Index of grid row / plane q for the input ring: periodic axes wrap (up to
// two cells beyond a face), other axes clamp (the rules that replace those
// values are applied by the consumers).
__device__ __forceinline__ int wrap_or_clamp(int q, int n, bool periodic) {
    if (periodic) return ((q % n) + n) % n;
    return min(max(q, 0), n - 1);
}

// LDS operations of this wave complete (before a barrier publishes them).
__device__ __forceinline__ void lds_done() {
    // vmcnt and expcnt at their maxima, lgkmcnt(0)
    __builtin_amdgcn_s_waitcnt(15 | (3 << 14) | (7 << 4));
}

// One LDS cell read (waited for in the same block) and one written, in
// assembly, by a producer wave between its direct-to-LDS loads: for an
// ordinary LDS access that might overlap a load in flight the compiler
// drains every load, which would empty the producer's pipeline.  (The cells
// these touch belong to loads already waited for.)
template <typename T>
__device__ __forceinline__ T lds_peek(const RD_LDS T* p) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 2, "cell size");
    uint32_t v;
#ifdef __HIP_DEVICE_COMPILE__
    const uint32_t addr = uint32_t(reinterpret_cast<uintptr_t>(p));
    if constexpr (sizeof(T) == 4)
        asm volatile("ds_read_b32 %0, %1\n\ts_waitcnt lgkmcnt(0)" : "=v"(v) : "v"(addr));
    else
        asm volatile("ds_read_u16 %0, %1\n\ts_waitcnt lgkmcnt(0)" : "=v"(v) : "v"(addr));
#else
    (void)p;
    v = 0;
#endif
    T r;
    __builtin_memcpy(&r, &v, sizeof(T));
    return r;
}
template <typename T>
__device__ __forceinline__ void lds_poke(RD_LDS T* p, T x) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 2, "cell size");
    uint32_t v = 0;
    __builtin_memcpy(&v, &x, sizeof(T));
#ifdef __HIP_DEVICE_COMPILE__
    const uint32_t addr = uint32_t(reinterpret_cast<uintptr_t>(p));
    if constexpr (sizeof(T) == 4) asm volatile("ds_write_b32 %0, %1" : : "v"(addr), "v"(v));
    else asm volatile("ds_write_b16 %0, %1" : : "v"(addr), "v"(v));
#else
    (void)p;
#endif
}

template <class M, int NCH, int BY, int WC, int D>
__device__ __forceinline__ void lds2_producer(const StepArgs& a, RD_LDS float* iring, int yb, int z0, int z1) {
    using R = Lds2Ring<M::NF, NCH, BY, D>;
    constexpr int NF = M::NF, IROWS = R::IROWS, TXT = R::TXT;
    const int lane = threadIdx.x & 63;
    int ridx[NF][IROWS];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int j = 0; j < IROWS; ++j)
            ridx[f][j] = wrap_or_clamp(yb - 2 + j, a.ny, a.bck[f][2] == BC_PERIODIC);
    auto issue = [&](int slot, int p) __attribute__((always_inline)) {
        RD_LDS float* base_l = iring + slot * R::ISLOT;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const int pz = wrap_or_clamp(p, a.nz, a.bck[f][4] == BC_PERIODIC);
            const RD_GLOBAL float* base = gload_ptr<float>(a.in[f]) + (long long)pz * a.plane + lane * 4;
#pragma unroll
            for (int j = 0; j < IROWS; ++j)
#pragma unroll
                for (int c = 0; c < NCH; ++c)
                    __builtin_amdgcn_global_load_lds(
                        base + (long long)ridx[f][j] * a.pitch + c * 256,
                        (RD_LDS void*)(base_l + (f * IROWS + j) * TXT + c * 256), 16, 0, 0);
        }
    };
    // input planes z0-2 .. z1+1; plane p lives in slot (p - z0 + 2) % D
    const int p_first = z0 - 2, p_last = z1 + 1;
    for (int k = 0; k < D - 1 && p_first + k <= p_last; ++k) issue(k, p_first + k);
    int slot_next = (D - 1) % D;        // slot of plane q + D - 2 at iteration q = z0 - 1
    for (int q = z0 - 1; q <= z1 + 1; ++q) {
        if (q <= z1) vm_wait_steps<R::CH, D - 4>(min(D - 4, z1 - q));   // plane q+1 complete
        ring_barrier();
        if (q + D - 2 <= p_last) issue(slot_next, q + D - 2);
        slot_next = slot_next + 1 == D ? 0 : slot_next + 1;
    }
}

// Mid-ring row for output neighbour row yn (grid index) of a tile starting at
// yb, by the y face rules; cst: use value v.
struct MidSrc { int idx; int cst; float v; };

__device__ __forceinline__ MidSrc mid_src(int q, int n, int base, int klo, int khi, float vlo, float vhi) {
    if (q >= 0 && q < n) return MidSrc{q - base, 0, 0.f};
    const int k = q < 0 ? klo : khi;
    if (k == BC_PERIODIC) return MidSrc{q - base, 0, 0.f};
    if (k == BC_MIRROR) return MidSrc{(q < 0 ? 0 : n - 1) - base, 0, 0.f};
    return MidSrc{0, 1, q < 0 ? vlo : vhi};
}

template <class M, int NCH, int BY, int WC, int D>
__device__ __forceinline__ void lds2_consumer(const StepArgs& a, const RD_LDS float* iring, RD_LDS float* mring, int cw,
                                              int yb, int z0, int z1) {
    static_assert(!M::SOURCES && M::NO == M::NF, "point sources and extra fields are not blocked");
    using R = Lds2Ring<M::NF, NCH, BY, D>;
    constexpr int NF = M::NF, NO = M::NO, TXT = R::TXT, IROWS = R::IROWS, MROWS = R::MROWS;
    constexpr int MPW = (MROWS + WC - 1) / WC;     // mid rows per wave (the last ones may idle)
    constexpr int OPW = (BY + WC - 1) / WC;        // output rows per wave
    const int lane = threadIdx.x & 63;
    int xsl[NF], xsr[NF];
    (void)x_sides<M, true>(a, 0, TXT, true, xsl, xsr);
    bool any_held = false, in_fix = false;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        any_held = any_held || a.held[f] != 0 || a.out_held[f] != 0;
        for (int k = 0; k < 6; ++k) in_fix = in_fix || a.bck[f][k] == BC_GHOST || a.bck[f][k] == BC_HELD;
    }
    in_fix = in_fix || any_held;

    // x neighbours of lane values v (chunks of 4 per lane) by the x face rules
    auto xnb = [&](int f, const float (&v)[NCH][4], int c, float& left, float& right) __attribute__((always_inline)) {
        float fl, fr;
        if (c > 0) fl = lane_from_left_wrap(v[c - 1][3]);
        else if (xsl[f] == XS_ROT) fl = lane_from_left_wrap(v[NCH - 1][3]);
        else fl = xsl[f] == XS_OWN ? v[0][0] : a.bcv[f][0];
        if (c < NCH - 1) fr = lane_from_right_wrap(v[c + 1][0]);
        else if (xsr[f] == XS_ROT) fr = lane_from_right_wrap(v[0][0]);
        else fr = xsr[f] == XS_OWN ? v[NCH - 1][3] : a.bcv[f][1];
        left = lane_from_left(v[c][3], fl);
        right = lane_from_right(v[c][0], fr);
    };
    auto ld4 = [&](const RD_LDS float* p, float (&o)[4]) __attribute__((always_inline)) { lds_ld4(p, o); };

    int islot0 = 0;              // input slot of plane q-1 at iteration q (plane z0-2 is slot 0)
    int mslot = 0;               // mid slot of plane q (mid plane z0-1 is slot 0)
    for (int q = z0 - 1; q <= z1 + 1; ++q) {
        lds_done();
        ring_barrier();
        // ---- mid plane q on rows yb-1 .. yb+BY (mid row m = grid row yb-1+m)
        if (q <= z1) {
            const int sm = islot0, s0 = islot0 + 1 == D ? 0 : islot0 + 1, sp = s0 + 1 == D ? 0 : s0 + 1;
            const RD_LDS float* Im = iring + sm * R::ISLOT;
            const RD_LDS float* I0 = iring + s0 * R::ISLOT;
            const RD_LDS float* Ip = iring + sp * R::ISLOT;
            RD_LDS float* Mq = mring + mslot * R::MSLOT;
#pragma unroll
            for (int k = 0; k < MPW; ++k) {
                const int m = cw + k * WC;
                if (m < MROWS) {
                    const int y = yb - 1 + m;
                    float v0[NF][3][NCH][4], vm[NF][NCH][4], vp[NF][NCH][4];
#pragma unroll
                    for (int f = 0; f < NF; ++f)
#pragma unroll
                        for (int c = 0; c < NCH; ++c) {
#pragma unroll
                            for (int r = 0; r < 3; ++r)
                                ld4(I0 + (f * IROWS + m + r) * TXT + c * 256 + lane * 4, v0[f][r][c]);
                            ld4(Im + (f * IROWS + m + 1) * TXT + c * 256 + lane * 4, vm[f][c]);
                            ld4(Ip + (f * IROWS + m + 1) * TXT + c * 256 + lane * 4, vp[f][c]);
                        }
                    if (in_fix) {
                        // input values fixed by a rule (ghost or held rows, planes, x faces)
#pragma unroll
                        for (int f = 0; f < NF; ++f) {
                            const int* kk = a.bck[f];
                            const float* vv = a.bcv[f];
                            const Src pm = resolve_axis(q - 1, a.nz, kk[4], kk[5], vv[4], vv[5]);
                            const Src p0 = resolve_axis(q, a.nz, kk[4], kk[5], vv[4], vv[5]);
                            const Src pp = resolve_axis(q + 1, a.nz, kk[4], kk[5], vv[4], vv[5]);
                            Src ry[3];
#pragma unroll
                            for (int r = 0; r < 3; ++r) ry[r] = resolve_axis(y - 1 + r, a.ny, kk[2], kk[3], vv[2], vv[3]);
#pragma unroll
                            for (int c = 0; c < NCH; ++c) {
                                const int xl = c * 256 + lane * 4;
#pragma unroll
                                for (int r = 0; r < 3; ++r) fix_row<4>(a, f, p0, ry[r], xl, v0[f][r][c]);
                                fix_row<4>(a, f, pm, ry[1], xl, vm[f][c]);
                                fix_row<4>(a, f, pp, ry[1], xl, vp[f][c]);
                            }
                        }
                    }
                    Nb n[NF][NCH][4];
#pragma unroll
                    for (int f = 0; f < NF; ++f) {
                        float cen[NCH][4];
#pragma unroll
                        for (int c = 0; c < NCH; ++c)
#pragma unroll
                            for (int i = 0; i < 4; ++i) cen[c][i] = v0[f][1][c][i];
#pragma unroll
                        for (int c = 0; c < NCH; ++c) {
                            float left, right;
                            xnb(f, cen, c, left, right);
#pragma unroll
                            for (int i = 0; i < 4; ++i) {
                                Nb& t = n[f][c][i];
                                t.c = cen[c][i];
                                t.xm = i > 0 ? cen[c][i - 1] : left;
                                t.xp = i < 3 ? cen[c][i + 1] : right;
                                t.ym = v0[f][0][c][i];
                                t.yp = v0[f][2][c][i];
                                t.zm = vm[f][c][i];
                                t.zp = vp[f][c][i];
                            }
                        }
                    }
#pragma unroll
                    for (int c = 0; c < NCH; ++c) {
                        const int xl = c * 256 + lane * 4;
                        float o[NO][4];
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            Nb ni[NF];
#pragma unroll
                            for (int f = 0; f < NF; ++f) ni[f] = n[f][c][i];
                            const float e[NO] = {};
                            float oi[NO];
                            M::cell(a, ni, 0.f, false, e, oi);
#pragma unroll
                            for (int s = 0; s < NO; ++s) o[s][i] = any_held ? held_out(a, s, xl + i, y, q, oi[s]) : oi[s];
                        }
#pragma unroll
                        for (int s = 0; s < NO; ++s)
                            lds_st4(Mq + (s * MROWS + m) * TXT + c * 256 + lane * 4, o[s][0], o[s][1], o[s][2], o[s][3]);
                    }
                }
            }
        }
        // ---- output plane z = q-2 on rows yb .. yb+BY-1, from mid planes z-1, z, z+1
        const int z = q - 2;
        if (z >= z0) {
            const int ms_z = (mslot + 2) & 3;          // mid plane q-2
            const int ms_m = (mslot + 1) & 3;          // mid plane q-3
            const int ms_p = (mslot + 3) & 3;          // mid plane q-1
#pragma unroll
            for (int rr = 0; rr < OPW; ++rr) {
                const int r = cw + rr * WC;
                if (r >= BY) break;
                const int y = yb + r;
                float v0[NF][3][NCH][4], vm[NF][NCH][4], vp[NF][NCH][4];
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const int* kk = a.bck[f];
                    const float* vv = a.bcv[f];
                    // mid rows y-1, y, y+1 and mid planes z-1, z+1 by the face rules
                    MidSrc ry[3];
#pragma unroll
                    for (int t = 0; t < 3; ++t) ry[t] = mid_src(y - 1 + t, a.ny, yb - 1, kk[2], kk[3], vv[2], vv[3]);
                    const MidSrc pzm = mid_src(z - 1, a.nz, z - 1, kk[4], kk[5], vv[4], vv[5]);
                    const MidSrc pzp = mid_src(z + 1, a.nz, z - 1, kk[4], kk[5], vv[4], vv[5]);
                    // pzm.idx / pzp.idx: 0 = plane z-1, 1 = plane z, 2 = plane z+1
                    const RD_LDS float* Mz = mring + ms_z * R::MSLOT + f * MROWS * TXT;
                    const RD_LDS float* Mm = mring + (pzm.idx == 1 ? ms_z : ms_m) * R::MSLOT + f * MROWS * TXT;
                    const RD_LDS float* Mp = mring + (pzp.idx == 1 ? ms_z : ms_p) * R::MSLOT + f * MROWS * TXT;
#pragma unroll
                    for (int c = 0; c < NCH; ++c) {
#pragma unroll
                        for (int t = 0; t < 3; ++t) {
                            ld4(Mz + ry[t].idx * TXT + c * 256 + lane * 4, v0[f][t][c]);
                            if (ry[t].cst)
#pragma unroll
                                for (int i = 0; i < 4; ++i) v0[f][t][c][i] = ry[t].v;
                        }
                        ld4(Mm + ry[1].idx * TXT + c * 256 + lane * 4, vm[f][c]);
                        ld4(Mp + ry[1].idx * TXT + c * 256 + lane * 4, vp[f][c]);
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            if (pzm.cst) vm[f][c][i] = pzm.v;
                            if (pzp.cst) vp[f][c][i] = pzp.v;
                        }
                    }
                }
                Nb n[NF][NCH][4];
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    float cen[NCH][4];
#pragma unroll
                    for (int c = 0; c < NCH; ++c)
#pragma unroll
                        for (int i = 0; i < 4; ++i) cen[c][i] = v0[f][1][c][i];
#pragma unroll
                    for (int c = 0; c < NCH; ++c) {
                        float left, right;
                        xnb(f, cen, c, left, right);
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            Nb& t = n[f][c][i];
                            t.c = cen[c][i];
                            t.xm = i > 0 ? cen[c][i - 1] : left;
                            t.xp = i < 3 ? cen[c][i + 1] : right;
                            t.ym = v0[f][0][c][i];
                            t.yp = v0[f][2][c][i];
                            t.zm = vm[f][c][i];
                            t.zp = vp[f][c][i];
                        }
                    }
                }
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    const int xl = c * 256 + lane * 4;
                    float o[NO][4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        Nb ni[NF];
#pragma unroll
                        for (int f = 0; f < NF; ++f) ni[f] = n[f][c][i];
                        const float e[NO] = {};
                        float oi[NO];
                        M::cell(a, ni, 0.f, false, e, oi);
#pragma unroll
                        for (int s = 0; s < NO; ++s) o[s][i] = any_held ? held_out(a, s, xl + i, y, z, oi[s]) : oi[s];
                    }
                    if (y < a.ny) {
                        const long long idx = (long long)z * a.plane + (long long)y * a.pitch + xl;
#pragma unroll
                        for (int s = 0; s < NO; ++s) store_vec<StF32, 4>(a.out[s], idx, o[s]);
                    }
                }
            }
        }
        islot0 = islot0 + 1 == D ? 0 : islot0 + 1;
        mslot = (mslot + 1) & 3;
    }
}

template <class M, int NCH, int BY, int WC, int D>
__global__ __launch_bounds__(64 * (WC + 1)) void lds2_kernel(const StepArgs* __restrict__ pa) {
    using R = Lds2Ring<M::NF, NCH, BY, D>;
    static_assert(R::FITS, "ring shape does not fit");
    static_assert(M::WIND != WIND_CLOCK, "a clocked wind is not blocked in time");
    __shared__ __attribute__((aligned(16))) float iring[D * R::ISLOT];
    __shared__ __attribute__((aligned(16))) float mring[4 * R::MSLOT];
    const StepArgs& a = *pa;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const TileXYZ tc = tile_coords(a, xcd_tile(blockIdx.x, gridDim.x));
    const int yb = tc.y * BY;
    const int z0 = tc.z * a.cz;
    const int z1 = min(z0 + a.cz, a.nz);
    RD_LDS float* ib = (RD_LDS float*)&iring[0];
    RD_LDS float* mb = (RD_LDS float*)&mring[0];
    if (w == 0) lds2_producer<M, NCH, BY, WC, D>(a, ib, yb, z0, z1);
    else lds2_consumer<M, NCH, BY, WC, D>(a, ib, mb, w - 1, yb, z0, z1);
}

// ------------------------------------------------------------ batch table
// The batched launch (rd_tring.hpp, batched_tr_kernel) walks the (grid,
// tile) work items of many grids.  The host writes, before each tick, `meta`
// = {ngrids, total_items, ticket, finished, first_item[0 .. ngrids]} (the two
// counters zero) and one entry per grid:
// its step arguments for both parities (tiled for that kernel), model,
// parity of the current state, steps left.

struct BatchEntry {
    StepArgs args[2];     // by input parity
    int model;            // 0 diffusion (1 species), 1 Brusselator
    int ntiles;
    int first_item;
    int parity;           // parity of the current state at tick start
    long long steps_left; // at tick start
};

// ------------------------------------------------------------- reductions

template <class S>
__global__ __launch_bounds__(256) void reduce_partial(const void* f, int nx, int ny, int nz,
                                                      int pitch, long long plane, double* part) {
    double s = 0.0, q = 0.0;
    const long long rows = (long long)ny * nz;
    for (long long row = blockIdx.x; row < rows; row += gridDim.x) {
        const long long base = (row / ny) * plane + (row % ny) * (long long)pitch;
        for (int x = threadIdx.x; x < nx; x += 256) {
            const double v = load1<S>(f, base + x);
            s += v;
            q += v * v;
        }
    }
    __shared__ double ss[256], sq[256];
    ss[threadIdx.x] = s;
    sq[threadIdx.x] = q;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) {
            ss[threadIdx.x] += ss[threadIdx.x + k];
            sq[threadIdx.x] += sq[threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = ss[0];
        part[2 * blockIdx.x + 1] = sq[0];
    }
}

#ifdef RD_DEFINE_ENGINE_KERNELS   // non-template kernels: one definition, in the engine
__global__ __launch_bounds__(256) void reduce_final(const double* part, int n, double h3, double* out) {
    double s = 0.0, q = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        s += part[2 * i];
        q += part[2 * i + 1];
    }
    __shared__ double ss[256], sq[256];
    ss[threadIdx.x] = s;
    sq[threadIdx.x] = q;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) {
            ss[threadIdx.x] += ss[threadIdx.x + k];
            sq[threadIdx.x] += sq[threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = ss[0] * h3;
        out[1] = sq[0] * h3;
    }
}

#endif

// ------------------------------------------------------ layout conversion

// dense [nz][ny][nx] of transfer type Src -> padded storage S
template <class S, class Src>
__global__ __launch_bounds__(256) void pack_kernel(const void* src, void* dst, int nx, int ny, int nz,
                                                   int pitch, long long plane) {
    const long long n = (long long)nx * ny * nz;
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const long long x = i % nx, r = i / nx;
        const long long y = r % ny, z = r / ny;
        const float v = Src::up(static_cast<const typename Src::T*>(src)[i]);
        static_cast<typename S::T*>(dst)[z * plane + y * pitch + x] = S::down(v);
    }
}

template <class S, typename DstT>
__global__ __launch_bounds__(256) void unpack_kernel(const void* src, DstT* dst, int nx, int ny, int nz,
                                                     int pitch, long long plane) {
    const long long n = (long long)nx * ny * nz;
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const long long x = i % nx, r = i / nx;
        const long long y = r % ny, z = r / ny;
        dst[i] = DstT(S::up(static_cast<const typename S::T*>(src)[z * plane + y * pitch + x]));
    }
}

#ifdef RD_DEFINE_ENGINE_KERNELS
// ----------------------------------------------------------- copy ceiling

// One 16-byte element per thread, streamed with non-temporal load/store:
// the read+write bandwidth ceiling a kernel can reach.
__global__ __launch_bounds__(256) void copy_kernel(const float4* __restrict__ src,
                                                   float4* __restrict__ dst, long long n4) {
    typedef float v4f __attribute__((ext_vector_type(4)));
    const long long i = blockIdx.x * 256LL + threadIdx.x;
    if (i < n4) {
        const v4f v = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(src) + i);
        __builtin_nontemporal_store(v, reinterpret_cast<v4f*>(dst) + i);
    }
}
#endif

}  // namespace rdk
