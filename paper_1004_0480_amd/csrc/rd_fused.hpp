// rd_fused.hpp -- the front model's step in one pass over HBM.
//
// The Cahn-Hilliard term of the front model needs the Laplacian twice: mu =
// gamma C^3 - eps C - kappa Lap(C), then M Lap(mu) (section 4.1 computes it
// with two kernels and a mu array in global memory).  Here one kernel reads
// A, B and C once and writes them once (24 bytes per cell-update in FP32
// instead of 36): mu is computed into LDS one plane ahead of the update and
// never leaves the chip.
//
// A workgroup owns an x tile of 128 cells (two per lane), rows [yb, yb+BY)
// and a z range [z0, z1).  One producer wave streams every plane into LDS
// rings with direct-to-LDS loads: A and B with one halo row on each side, C
// with two (mu is needed one row beyond the output rows), each row the tile
// plus one 16-byte unit on each side (the x halo).  Per plane q, after one
// barrier:
//   - WM waves compute mu of plane q+2 on rows yb-1 .. yb+BY and columns
//     x0-1 .. x0+128 from C planes q+1 .. q+3 into a ring of four LDS mu
//     planes;
//   - WU waves update plane q of A, B, C from the input ring (plane q and the
//     centre rows of q-1, q, q+1, kept in registers) and mu planes q-1 ..
//     q+1, computed in earlier iterations.
// Every value goes through the same arithmetic as the two-pass plans
// (ChemPotential::mu, lapf, FrontCH::rates), and mu is FP32 as the mu array
// is, so the fused step gives the same values as the two passes (a Fickian
// term of C and a redissolution term that are zero are not formed, which can
// change only the sign of a zero).  mu takes mirror ghosts on every face (the boundary rule applied
// again before the second Laplacian); C, A and B their own face rules.
#pragma once

#include "rd_fch_cfg.hpp"

namespace rdk {

// Two input rings: C is read on planes q .. q+3 at iteration q (the
// chemical potential of plane q+2 needs C one plane either side), A and B
// only on planes q and q+1 (the update of plane q), so the A/B ring has two
// slots fewer and both rings keep DC - 4 planes in flight.
template <class S, int BY, int DC>
struct Fch {
    using T = typename S::T;
    static constexpr int ES = int(sizeof(T));
    static constexpr int TX = kFchTile;            // cells of a row per workgroup
    static constexpr int HX = 16 / ES;             // halo cells per side: one 16-byte unit
    static constexpr int RW = TX + 2 * HX;         // cells per ring row: x0-HX .. x0+TX+HX-1
    static constexpr int NU = RW / HX;             // 16-byte units per ring row
    static constexpr int RA = BY + 2;              // ring rows of A and B: grid rows yb-1 .. yb+BY
    static constexpr int RC = BY + 4;              // ring rows of C: grid rows yb-2 .. yb+BY+1
    static constexpr int DAB = DC - 2;             // slots of the A/B ring
    static constexpr int SLOTC = RC * RW;          // cells per C slot
    static constexpr int SLOTAB = 2 * RA * RW;     // cells per A/B slot
    static constexpr int SLOTC_W = SLOTC * ES / 4, SLOTAB_W = SLOTAB * ES / 4;   // in 4-byte words
    static constexpr int MW = TX + 4;              // mu row: x0-2 .. x0+TX+1 (FP32)
    static constexpr int MROWS = BY + 2;           // mu rows: grid rows yb-1 .. yb+BY
    static constexpr int MSLOT = MROWS * MW;       // floats per mu plane
    static_assert(NU <= 64 && RW * ES % 16 == 0 && MW * 4 % 16 == 0 && DC >= 5, "ring layout");
    // ring row of field f's row j: A and B in the A/B ring, C in its own
    static __host__ __device__ constexpr int row0(int f) { return f == 2 ? 0 : f * RA; }
    // grid row of ring row 0 of field f is yb - lead(f)
    static __host__ __device__ constexpr int lead(int f) { return f == 2 ? 2 : 1; }
};

// The producer issues "steps": step k loads C plane z0-2+k (planes z0-2 ..
// z1+1 exist) into C slot k mod DC and A/B plane z0-4+k (planes z0-1 .. z1)
// into A/B slot (k-3) mod DAB.  Both planes of step k are first read at
// iteration q = z0-5+k (C plane q+3, A/B plane q+1).  After barrier q the
// slots of C and A/B plane q-1 are free and take step q+DC+1-z0; before it,
// step q+5-z0 must have landed, with the DC-5 steps issued after it still in
// flight.
template <class S, int BY, int DC>
__device__ __forceinline__ void fch_producer(const StepArgs& a, RD_LDS float* ring_c, RD_LDS float* ring_ab,
                                             int x0, int yb, int z0, int z1) {
#ifndef __HIP_DEVICE_COMPILE__
    (void)a, (void)ring_c, (void)ring_ab, (void)x0, (void)yb, (void)z0, (void)z1;
#else
    using F = Fch<S, BY, DC>;
    using T = typename F::T;
    const int lane = threadIdx.x & 63;
    // column (from the row start) of this lane's 16-byte unit, per field: the
    // tile and its halo units; at the grid's x faces a halo unit is loaded
    // only for a periodic axis (the unit holding cell nx-1 on the left, cells
    // 0 .. HX-1 on the right), else the face rule supplies the value
    int col[3];
    bool act[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        const bool per = a.bck[f][0] == BC_PERIODIC;
        col[f] = x0 - F::HX + lane * F::HX;
        act[f] = lane < F::NU;
        if (lane == 0 && x0 == 0) {
            col[f] = (a.nx - 1) / F::HX * F::HX;
            act[f] = per;
        }
        if (lane == F::NU - 1 && x0 + F::TX >= a.nx) {
            col[f] = 0;
            act[f] = per;
        }
    }
    // grid row of every ring row by the y face rules (fixed values are
    // applied by the computing waves)
    int rab[2][F::RA], rc[F::RC];
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
        for (int j = 0; j < F::RA; ++j)
            rab[f][j] = resolve_axis(yb - 1 + j, a.ny, a.bck[f][2], a.bck[f][3], a.bcv[f][2], a.bcv[f][3]).idx;
#pragma unroll
    for (int j = 0; j < F::RC; ++j)
        rc[j] = resolve_axis(yb - 2 + j, a.ny, a.bck[2][2], a.bck[2][3], a.bcv[2][2], a.bcv[2][3]).idx;
    // byte offset, within a plane, of this lane's 16-byte unit of every ring
    // row (the rows are the same on every plane)
    unsigned oc[F::RC], oab[2][F::RA];
#pragma unroll
    for (int j = 0; j < F::RC; ++j) oc[j] = unsigned(((long long)rc[j] * a.pitch + col[2]) * F::ES);
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
        for (int j = 0; j < F::RA; ++j) oab[f][j] = unsigned(((long long)rab[f][j] * a.pitch + col[f]) * F::ES);
    const long long pbytes = a.plane * F::ES;
    const int last_c = z1 + 3 - z0, first_ab = 3, last_ab = z1 + 4 - z0;   // steps that load
    auto count = [&](int k) __attribute__((always_inline)) {
        return (k >= 0 && k <= last_c ? F::RC : 0) + (k >= first_ab && k <= last_ab ? 2 * F::RA : 0);
    };
    // plane z of field f (the z face rules apply outside the grid)
    auto plane_of = [&](int f, int p) __attribute__((always_inline)) {
        const int pz = unsigned(p) < unsigned(a.nz)
                           ? p
                           : resolve_axis(p, a.nz, a.bck[f][4], a.bck[f][5], a.bcv[f][4], a.bcv[f][5]).idx;
        return (const RD_GLOBAL char*)a.in[f] + pz * pbytes;
    };
    // steps are issued in order, so their slots advance by one each
    int slot_c = 0, slot_ab = 0;
    auto issue = [&](int k) __attribute__((always_inline)) {
        if (k <= last_c) {
            RD_LDS T* sl = (RD_LDS T*)(ring_c + slot_c * F::SLOTC_W);
            const RD_GLOBAL char* base = plane_of(2, z0 - 2 + k);
#pragma unroll
            for (int j = 0; j < F::RC; ++j)
                if (act[2])
                    __builtin_amdgcn_global_load_lds((const RD_GLOBAL void*)(base + oc[j]),
                                                     (RD_LDS void*)(sl + j * F::RW), 16, 0, 0);
        }
        slot_c = slot_c + 1 == DC ? 0 : slot_c + 1;
        if (k >= first_ab && k <= last_ab) {
            RD_LDS T* sl = (RD_LDS T*)(ring_ab + slot_ab * F::SLOTAB_W);
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                const RD_GLOBAL char* base = plane_of(f, z0 - 4 + k);
#pragma unroll
                for (int j = 0; j < F::RA; ++j)
                    if (act[f])
                        __builtin_amdgcn_global_load_lds((const RD_GLOBAL void*)(base + oab[f][j]),
                                                         (RD_LDS void*)(sl + (f * F::RA + j) * F::RW), 16, 0, 0);
            }
            slot_ab = slot_ab + 1 == F::DAB ? 0 : slot_ab + 1;
        }
    };
    for (int k = 0; k < DC - 2; ++k) issue(k);
    // in the steady state every step loads C and A/B
    constexpr int STEADY = (DC - 5) * (F::RC + 2 * F::RA) < 63 ? (DC - 5) * (F::RC + 2 * F::RA) : 63;
    for (int q = z0 - 3; q < z1; ++q) {
        // step q+5-z0 complete: the steps issued after it may stay in flight
        const int need = q + 5 - z0;
        if (need + 1 >= first_ab && need + DC - 5 <= last_c) {
            vm_wait_imm<STEADY>();
        } else {
            int after = 0;
#pragma unroll
            for (int j = 1; j <= DC - 5; ++j) after += count(need + j);
            vm_wait_count<0, 63>(min(after, 63));
        }
        ring_barrier();
        issue(q + DC + 1 - z0);
    }
#endif
}

// The computing waves, in two roles: WU waves update A, B and C on BY/WU rows
// each, WM waves compute the chemical potential (its rows dealt round-robin;
// the last of them also computes the columns x0-1 and x0+TX of every mu row,
// one lane per row and side).  XF: the tile touches an x face of the grid
// (x0 = 0 or the row ends in it), so x neighbours there follow the face
// rules; without it every x neighbour comes from the tile or its halo.
// Within the plane loop each phase runs in a FIX variant (boundary rules
// replace loaded values, held outputs) only where a row or plane of it is
// fixed, so the common case carries no boundary logic.
template <class S, int BY, int WU, int WM, int DC, bool XF>
struct FchConsumer {
    using F = Fch<S, BY, DC>;
    static constexpr int DAB = F::DAB;
    using T = typename F::T;
    static constexpr int RY = BY / WU, MPW = (F::MROWS + WM - 1) / WM;
    static constexpr int HX = F::HX, TX = F::TX, RW = F::RW, MW = F::MW;
    static constexpr int STORE_ANY = 0, STORE_PLAIN = 1, STORE_SR = 2;   // update's store forms
    typedef float v2f __attribute__((ext_vector_type(2)));

    const StepArgs& a;
    const CellConst k;
    const RD_LDS T* ring_c;
    const RD_LDS T* ring_ab;
    RD_LDS float* mring;
    int lane, x0, yb, xl;
    // XF: the x face rules of the three fields at this tile (kind and value
    // on each side), fixed for the march, where the tile meets each face, and
    // whether this lane's cells are the grid's last; the LDS cell of x0-1
    int fk[3][2];
    float fv[3][2];
    bool lface, rface, last0, last1;
    int hlo;
    __device__ __forceinline__ FchConsumer(const StepArgs& a_, const RD_LDS float* ring_c_w,
                                           const RD_LDS float* ring_ab_w, RD_LDS float* mring_, int x0_, int yb_)
        : a(a_), k(a_), ring_c((const RD_LDS T*)ring_c_w), ring_ab((const RD_LDS T*)ring_ab_w), mring(mring_),
          lane(threadIdx.x & 63), x0(x0_), yb(yb_), xl(x0_ + 2 * (threadIdx.x & 63)) {
        lface = rface = last0 = last1 = false;
        hlo = HX - 1;
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                fk[f][side] = BC_MIRROR;
                fv[f][side] = 0.f;
            }
        if constexpr (XF) {
            lface = x0 == 0;
            rface = x0 + TX >= a.nx;
            last0 = xl == a.nx - 1;
            last1 = xl + 1 == a.nx - 1;
            // at the left face of a periodic axis the halo holds the 16-byte
            // unit with cell nx-1
            hlo = lface ? (a.nx - 1) % HX : HX - 1;
#pragma unroll
            for (int f = 0; f < 3; ++f)
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    fk[f][side] = a.bck[f][side];
                    fv[f][side] = vcopy(a.bcv[f][side]);
                }
        }
    }
    // mu from C and Lap(C), and the rates of the front model
    __device__ __forceinline__ float mu_of(float c, float lc) const { return ChemPotential::mu(k, c, lc); }
    __device__ __forceinline__ void rates(float A, float B, float C, float la, float lb, float lc, float lmu,
                                          float q, float (&o)[3]) const {
        FrontCH::rates(k, A, B, C, la, lb, lc, lmu, q, o);
    }

    // C slot s, A/B slot s, and the slot base of field f (C slot sc or A/B slot sab)
    __device__ __forceinline__ const RD_LDS T* cslot(int s) const { return ring_c + s * F::SLOTC; }
    __device__ __forceinline__ const RD_LDS T* abslot(int s) const { return ring_ab + s * F::SLOTAB; }
    static __device__ __forceinline__ const RD_LDS T* row(const RD_LDS T* P, int f, int j) {
        return P + (F::row0(f) + j) * RW;
    }
    // this lane's two cells of a ring row, as FP32
    __device__ __forceinline__ void rd2(const RD_LDS T* r, float (&o)[2]) const {
        const RD_LDS T* q = r + HX + 2 * lane;
        if constexpr (sizeof(T) == 4) {
            const v2f t = *(const RD_LDS v2f*)q;
            o[0] = t.x;
            o[1] = t.y;
        } else {
            const unsigned t = *(const RD_LDS unsigned*)q;
            o[0] = S::up(T(t & 0xffffu));
            o[1] = S::up(T(t >> 16));
        }
    }
    static __device__ __forceinline__ float rd1(const RD_LDS T* r, int off) { return S::up(r[off]); }
    __device__ __forceinline__ RD_LDS float* mrow(int p, int m) const { return mring + (p & 3) * F::MSLOT + m * MW; }
    __device__ __forceinline__ void mrd2(const RD_LDS float* r, float (&o)[2]) const {
        const v2f t = *(const RD_LDS v2f*)(r + 2 + 2 * lane);
        o[0] = t.x;
        o[1] = t.y;
    }
    __device__ __forceinline__ Src ysrc(int f, int y) const {
        return resolve_axis(y, a.ny, a.bck[f][2], a.bck[f][3], a.bcv[f][2], a.bcv[f][3]);
    }
    __device__ __forceinline__ Src zsrc(int f, int z) const {
        return resolve_axis(z, a.nz, a.bck[f][4], a.bck[f][5], a.bcv[f][4], a.bcv[f][5]);
    }
    static __device__ __forceinline__ void fix1(const StepArgs& a, int f, Src pz, Src py, int x, float& v) {
        float t[1] = {v};
        fix_row<1>(a, f, pz, py, x, t);
        v = t[0];
    }
    // LDS cell of x0-1
    __device__ __forceinline__ int hl_off() const { return hlo; }
    __device__ __forceinline__ bool near(int p) const { return p <= 0 || p >= a.nz - 1; }

    // x neighbours of this lane's two cells (values v; halo cells hl = x0-1,
    // hr = x0+TX), by the x face rules of field f at the grid's faces
    __device__ __forceinline__ void xnb(int f, const float (&v)[2], float hl, float hr, float (&xm)[2],
                                        float (&xp)[2]) const {
        float fill = hl;
        if constexpr (XF) {
            const int kl = fk[f][0];
            if (lface && kl != BC_PERIODIC) fill = kl == BC_MIRROR ? v[0] : fv[f][0];
        }
        xm[0] = lane_from_left(v[1], fill);
        xm[1] = v[0];
        xp[0] = v[1];
        xp[1] = lane_from_right(v[0], hr);
        if constexpr (XF) {
            if (rface) {
                const int kr = fk[f][1];
                const float g = fv[f][1];
                if (last0) xp[0] = kr == BC_MIRROR ? v[0] : kr == BC_PERIODIC ? hr : g;
                if (last1) xp[1] = kr == BC_MIRROR ? v[1] : kr == BC_PERIODIC ? hr : g;
            }
        }
    }

    // ---- chemical potential ------------------------------------------------

    // C around this lane's two cells of mu row m: the five points of the
    // Laplacian from C planes p-1 (P1), p (P2), p+1 (P3), and the row's x
    // halo cells
    struct MuIn {
        float c[2], cym[2], cyp[2], czm[2], czp[2], hl, hr;
    };
    __device__ __forceinline__ void mu_read(int m, const RD_LDS T* P1, const RD_LDS T* P2, const RD_LDS T* P3,
                                            MuIn& in) const {
        const int j = m + 1;                       // C ring row of grid row yb - 1 + m
        const RD_LDS T* rc = row(P2, 2, j);
        rd2(rc, in.c);
        rd2(row(P2, 2, j - 1), in.cym);
        rd2(row(P2, 2, j + 1), in.cyp);
        rd2(row(P1, 2, j), in.czm);
        rd2(row(P3, 2, j), in.czp);
        in.hl = rd1(rc, hl_off());
        in.hr = rd1(rc, HX + TX);
    }
    // mu of plane p, row m, at this lane's two cells
    template <bool FIX>
    __device__ __forceinline__ v2f mu_cells(int p, int m, MuIn in) const {
        if constexpr (FIX) {
            const int gm = yb - 1 + m;
            const Src y0 = ysrc(2, gm), ym = ysrc(2, gm - 1), yp = ysrc(2, gm + 1);
            const Src pm = zsrc(2, p - 1), p0 = zsrc(2, p), pp = zsrc(2, p + 1);
            fix_row<2>(a, 2, p0, y0, xl, in.c);
            fix_row<2>(a, 2, p0, ym, xl, in.cym);
            fix_row<2>(a, 2, p0, yp, xl, in.cyp);
            fix_row<2>(a, 2, pm, y0, xl, in.czm);
            fix_row<2>(a, 2, pp, y0, xl, in.czp);
            fix1(a, 2, p0, y0, x0 == 0 ? a.nx - 1 : x0 - 1, in.hl);
            fix1(a, 2, p0, y0, x0 + TX, in.hr);
        }
        float xm[2], xp[2];
        xnb(2, in.c, in.hl, in.hr, xm, xp);
        v2f mu;
        const Nb n0{in.c[0], xm[0], xp[0], in.cym[0], in.cyp[0], in.czm[0], in.czp[0]};
        const Nb n1{in.c[1], xm[1], xp[1], in.cym[1], in.cyp[1], in.czm[1], in.czp[1]};
        mu.x = mu_of(in.c[0], lapf(n0, k, 3));
        mu.y = mu_of(in.c[1], lapf(n1, k, 3));
        return mu;
    }

    // mu at the columns x0-1 and x0+TX of every mu row: lane 2m + s takes mu
    // row m, side s (0: x0-1, 1: x0+TX).  Where this lane's cell lies, fixed
    // for the whole march:
    struct ColAt {
        int m, j, eo, xe;
        bool want;      // the cell exists and this tile needs it
        bool rface;     // x0+TX = nx-1: its right neighbour is the face rule
    };
    __device__ __forceinline__ ColAt col_at() const {
        ColAt c;
        c.m = lane >> 1;
        const int side = lane & 1;
        const int gm = yb - 1 + c.m;
        c.want = c.m < F::MROWS && gm >= 0 && gm < a.ny && (side ? x0 + TX < a.nx : x0 > 0);
        c.j = c.want ? c.m + 1 : 1;
        c.eo = side ? HX + TX : HX - 1;
        c.xe = side ? x0 + TX : x0 - 1;
        // (a tile of one cell follows this one, so this tile has no x face
        // itself; a periodic x axis is refused for such widths)
        c.rface = x0 + TX + 1 == a.nx && side;
        return c;
    }
    struct ColIn {
        float e, el, er, eym, eyp, ezm, ezp;
    };
    __device__ __forceinline__ void col_read(const ColAt& c, const RD_LDS T* P1, const RD_LDS T* P2,
                                             const RD_LDS T* P3, ColIn& in) const {
        const RD_LDS T* rc = row(P2, 2, c.j);
        in.e = rd1(rc, c.eo);
        in.el = rd1(rc, c.eo - 1);
        in.er = rd1(rc, c.eo + 1);
        in.eym = rd1(row(P2, 2, c.j - 1), c.eo);
        in.eyp = rd1(row(P2, 2, c.j + 1), c.eo);
        in.ezm = rd1(row(P1, 2, c.j), c.eo);
        in.ezp = rd1(row(P3, 2, c.j), c.eo);
    }
    template <bool FIX>
    __device__ __forceinline__ float col_cell(int p, const ColAt& c, ColIn in, bool rmirror, float rval) const {
        if constexpr (FIX) {
            const int gm = yb - 1 + c.m;
            const Src y0 = ysrc(2, gm), ym = ysrc(2, gm - 1), yp = ysrc(2, gm + 1);
            const Src pm = zsrc(2, p - 1), p0 = zsrc(2, p), pp = zsrc(2, p + 1);
            fix1(a, 2, p0, y0, c.xe, in.e);
            fix1(a, 2, p0, y0, c.xe - 1, in.el);
            fix1(a, 2, p0, y0, c.xe + 1, in.er);
            fix1(a, 2, p0, ym, c.xe, in.eym);
            fix1(a, 2, p0, yp, c.xe, in.eyp);
            fix1(a, 2, pm, y0, c.xe, in.ezm);
            fix1(a, 2, pp, y0, c.xe, in.ezp);
        }
        if (c.rface) in.er = rmirror ? in.e : rval;
        const Nb ne{in.e, in.el, in.er, in.eym, in.eyp, in.ezm, in.ezp};
        return mu_of(in.e, lapf(ne, k, 3));
    }

    // one mu wave (index mw) over the z range: mu planes z0-1 .. z1
    __device__ __forceinline__ void run_mu(int mw, int z0, int z1) const {
        bool wfix = (a.held[2] & 3) != 0;
        // this wave's mu rows (clamped into the ring) and whether each lies in
        // the grid -- the same on every plane
        int mrows[MPW];
        bool rowok[MPW];
#pragma unroll
        for (int i = 0; i < MPW; ++i) {
            const int m = mw + i * WM, gm = yb - 1 + m;
            mrows[i] = min(m, F::MROWS - 1);
            rowok[i] = m < F::MROWS && gm >= 0 && gm < a.ny;
#pragma unroll
            for (int t = -1; t <= 1; ++t) wfix = wfix || ysrc(2, gm + t).cst != CST_NONE;
        }
        const bool columns = mw == WM - 1;
        if (columns)
            for (int m = 0; m < F::MROWS; ++m)
#pragma unroll
                for (int t = -1; t <= 1; ++t) wfix = wfix || ysrc(2, yb - 1 + m + t).cst != CST_NONE;
        const ColAt cat = col_at();
        const bool rmirror = a.bck[2][1] == BC_MIRROR;
        const float rval = a.bcv[2][1];
        // mu plane p = q + 2 exists for 0 <= p <= min(nz - 1, z1); C planes
        // p-1 .. p+1 take no z rule unless p <= 1 or p >= nz - 2
        const int q_last = min(a.nz - 1, z1) - 2, p_hi = a.nz - 2;
        int sq = DC - 1;                  // C slot of plane q (plane z0-2 is slot 0)
        // one plane: FX false compiles only the rule-free forms
        auto plane = [&](int q, auto fx) __attribute__((always_inline)) {
            constexpr bool FX = decltype(fx)::value;
            lds_done();
            ring_barrier();
            const int s1 = sq + 1 == DC ? 0 : sq + 1, s2 = s1 + 1 == DC ? 0 : s1 + 1, s3 = s2 + 1 == DC ? 0 : s2 + 1;
            const int p = q + 2;
            if (q >= -2 && q <= q_last) {
                const RD_LDS T* P1 = cslot(s1);
                const RD_LDS T* P2 = cslot(s2);
                const RD_LDS T* P3 = cslot(s3);
                // every LDS read first, then the arithmetic
                MuIn in[MPW];
                ColIn cin;
#pragma unroll
                for (int i = 0; i < MPW; ++i) mu_read(mrows[i], P1, P2, P3, in[i]);
                if (columns) col_read(cat, P1, P2, P3, cin);
                __builtin_amdgcn_sched_barrier(0);
                v2f mu[MPW];
                float mue = 0.f;
                if (FX && (wfix || p <= 1 || p >= p_hi)) {
#pragma unroll
                    for (int i = 0; i < MPW; ++i) mu[i] = mu_cells<true>(p, mrows[i], in[i]);
                    if (columns) mue = col_cell<true>(p, cat, cin, rmirror, rval);
                } else {
#pragma unroll
                    for (int i = 0; i < MPW; ++i) mu[i] = mu_cells<false>(p, mrows[i], in[i]);
                    if (columns) mue = col_cell<false>(p, cat, cin, rmirror, rval);
                }
#pragma unroll
                for (int i = 0; i < MPW; ++i)
                    if (rowok[i]) *(RD_LDS v2f*)(mrow(p, mrows[i]) + 2 + 2 * lane) = mu[i];
                if (columns && cat.want) mrow(p, cat.m)[(lane & 1) ? TX + 2 : 1] = mue;
            }
            sq = s1;
        };
        // mu planes 2 .. nz-3 (q = p - 2) take the rule-free forms unless the
        // wave has fixed rows
        const int qa = z0 - 3, qb = wfix ? qa : max(qa, min(z1, 0)), qc = wfix ? qa : max(qb, min(z1, p_hi - 2));
        for (int q = qa; q < qb; ++q) plane(q, std::true_type{});
        for (int q = qb; q < qc; ++q) plane(q, std::false_type{});
        for (int q = qc; q < z1; ++q) plane(q, std::true_type{});
    }

    // ---- update of A, B, C -------------------------------------------------

    // centre rows of the wave's output rows at plane p (slot P), rules applied
    template <bool FIX>
    __device__ __forceinline__ void centre(int r0, int p, const RD_LDS T* PC, const RD_LDS T* PAB,
                                           float (&c)[3][RY][2]) const {
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                rd2(row(f == 2 ? PC : PAB, f, r0 + r + F::lead(f)), c[f][r]);
                if constexpr (FIX) fix_row<2>(a, f, zsrc(f, p), ysrc(f, yb + r0 + r), xl, c[f][r]);
            }
    }

    // A, B, C of plane z on rows r0 ..: plane z (slot P0) for the y and x
    // neighbours, centre rows of z-1, z, z+1 from registers, mu planes.  CD
    // false: C has no Fickian term and there is no redissolution (k2 = 0),
    // so neither term is formed.  Stores (ST): STORE_PLAIN, no Runge-Kutta
    // combination and round-to-nearest; STORE_SR, no Runge-Kutta combination
    // and stochastic rounding to BF16 with the draws shared by lane pairs
    // (sr_pair); STORE_ANY, every other case, through the general store.

    // Stochastic rounding state of an update wave: step, key of species 0,
    // counter step from one plane to the next, and the species-2 words of the
    // next plane when the previous update drew them.
    struct SrState {
        unsigned n, key, dpc;
        unsigned carry[RY];
        bool have;
    };

    template <bool FIX, bool CD, int ST>
    __device__ __forceinline__ void update(int r0, int z, const RD_LDS T* PC, const RD_LDS T* PAB,
                                           const float (&cm)[3][RY][2], const float (&c0)[3][RY][2],
                                           const float (&cp)[3][RY][2], RD_GLOBAL T* const (&po)[3][RY],
                                           const bool (&rowst)[RY], const unsigned (&pc)[RY],
                                           SrState& sr) const {
        constexpr int NF = CD ? 3 : 2;               // fields with a Laplacian of their own
        const int hlo = hl_off();
        const int zm = max(z - 1, 0), zp = min(z + 1, a.nz - 1);
        // every LDS read of the plane is issued first, so that their
        // latencies overlap and one wait covers them
        float ym[NF][RY][2], yp[NF][RY][2], hl[NF][RY], hr[NF][RY];
        float mc[RY][2], mym[RY][2], myp[RY][2], mzm[RY][2], mzp[RY][2], ml[RY], mr[RY];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int y = yb + r0 + r;
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const int j = r0 + r + F::lead(f);
                const RD_LDS T* P0 = f == 2 ? PC : PAB;
                const RD_LDS T* rc = row(P0, f, j);
                rd2(row(P0, f, j - 1), ym[f][r]);
                rd2(row(P0, f, j + 1), yp[f][r]);
                hl[f][r] = rd1(rc, hlo);
                hr[f][r] = rd1(rc, HX + TX);
            }
            // mu: mirror ghosts on every face (rows and planes clamp)
            const int mi = y - (yb - 1);
            const RD_LDS float* m0 = mrow(z, mi);
            mrd2(m0, mc[r]);
            mrd2(mrow(z, max(y - 1, 0) - (yb - 1)), mym[r]);
            mrd2(mrow(z, min(y + 1, a.ny - 1) - (yb - 1)), myp[r]);
            mrd2(mrow(zm, mi), mzm[r]);
            mrd2(mrow(zp, mi), mzp[r]);
            ml[r] = m0[1];
            mr[r] = m0[TX + 2];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int y = yb + r0 + r;
            float lf[3][2];
            // no Laplacian of C: -0 is the exact identity of the addition it
            // enters, so that addition is dropped
            lf[2][0] = lf[2][1] = -0.f;
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                if constexpr (FIX) {
                    const Src pz = zsrc(f, z), y0 = ysrc(f, y);
                    fix_row<2>(a, f, pz, ysrc(f, y - 1), xl, ym[f][r]);
                    fix_row<2>(a, f, pz, ysrc(f, y + 1), xl, yp[f][r]);
                    fix1(a, f, pz, y0, x0 == 0 ? a.nx - 1 : x0 - 1, hl[f][r]);
                    fix1(a, f, pz, y0, x0 + TX, hr[f][r]);
                }
                float xm[2], xp[2];
                xnb(f, c0[f][r], hl[f][r], hr[f][r], xm, xp);
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    const Nb n{c0[f][r][i], xm[i], xp[i], ym[f][r][i], yp[f][r][i], cm[f][r][i], cp[f][r][i]};
                    lf[f][i] = lapf(n, k, f);
                }
            }
            float lmu[2];
            {
                float mlr = ml[r];
                if constexpr (XF) mlr = lface ? mc[r][0] : mlr;
                float xm[2], xp[2];
                xm[0] = lane_from_left(mc[r][1], mlr);
                xm[1] = mc[r][0];
                xp[0] = mc[r][1];
                xp[1] = lane_from_right(mc[r][0], mr[r]);
                if constexpr (XF) {
                    if (rface) {
                        if (last0) xp[0] = mc[r][0];
                        if (last1) xp[1] = mc[r][1];
                    }
                }
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    const Nb n{mc[r][i], xm[i], xp[i], mym[r][i], myp[r][i], mzm[r][i], mzp[r][i]};
                    lmu[i] = lapf(n, k, 3);
                }
            }
            float o[3][2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const float A = c0[0][r][i], B = c0[1][r][i], C = c0[2][r][i];
                const float q = CD ? (k.p[5] * A) * C : 0.f;
                float oi[3];
                rates(A, B, C, lf[0][i], lf[1][i], lf[2][i], lmu[i], q, oi);
#pragma unroll
                for (int s = 0; s < 3; ++s) o[s][i] = FIX ? held_out(a, s, xl + i, y, z, oi[s]) : oi[s];
            }
            if constexpr (ST == STORE_SR) {
                unsigned wd[3];
                sr_pair(pc[r], sr, r, wd);
                if (rowst[r]) {
#pragma unroll
                    for (int s = 0; s < 3; ++s)
                        *(RD_GLOBAL unsigned*)po[s][r] = unsigned(bf16_stochastic(o[s][0], wd[s] & 0xffffu)) |
                                                        (unsigned(bf16_stochastic(o[s][1], wd[s] >> 16)) << 16);
                }
            } else if (rowst[r]) {
                if constexpr (ST == STORE_PLAIN) {
#pragma unroll
                    for (int s = 0; s < 3; ++s) store_vec_at<S, 2>(po[s][r], o[s]);
                } else {
#pragma unroll
                    for (int s = 0; s < 3; ++s) store_field<S, 2>(a, s, xl, y, z, o[s]);
                }
            }
        }
    }

    // Random words of the lane's two cells for species 0, 1, 2 (bits 0-15 for
    // the first cell, 16-31 for the second), as the general store draws them:
    // the cells of a lane pair (four in a row, the first at a multiple of four
    // in the dense index) share counter c, and species s takes the call with
    // key key + s, the even lane its first word, the odd lane its second.  The
    // even lane makes the species-0 call and the odd lane the species-1 call,
    // each passing the word the other needs across the pair.  Species 2 is
    // drawn every other plane for two planes: the even lane makes this plane's
    // call (counter c), the odd lane the next plane's (c + dpc), and they swap
    // the words the other needs; the next plane takes its words from the
    // carry.  One and a half calls per lane and row instead of three.
    static __device__ __forceinline__ unsigned pair_swap(unsigned v) {
        // quad_perm [1, 0, 3, 2]: lanes 2i and 2i+1 exchange
        return unsigned(__builtin_amdgcn_mov_dpp(int(v), 0xB1, 0xF, 0xF, false));
    }
    __device__ __forceinline__ void sr_pair(unsigned c, SrState& sr, int r, unsigned (&wd)[3]) const {
        const bool odd = (threadIdx.x & 1) != 0;
        const PhiloxOut r01 = philox2x32_10(c, sr.n, sr.key + (odd ? 1u : 0u));
        const unsigned recv = pair_swap(odd ? r01.w0 : r01.w1);
        wd[0] = odd ? recv : r01.w0;
        wd[1] = odd ? r01.w1 : recv;
        if (sr.have) {
            wd[2] = sr.carry[r];
        } else {
            const PhiloxOut r2 = philox2x32_10(odd ? c + sr.dpc : c, sr.n, sr.key + 2u);
            const unsigned recv2 = pair_swap(odd ? r2.w0 : r2.w1);
            wd[2] = odd ? recv2 : r2.w0;          // this plane: the even lane's call
            sr.carry[r] = odd ? r2.w1 : recv2;    // next plane: the odd lane's call
        }
    }

    // one update wave (index uw) over the z range: planes z0 .. z1-1
    template <bool CD, int ST>
    __device__ __forceinline__ void run_update(int uw, int z0, int z1) const {
        const int r0 = uw * RY;
        bool wfix = false;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            wfix = wfix || (a.held[f] & 3) != 0;
#pragma unroll
            for (int r = -1; r <= RY; ++r) wfix = wfix || ysrc(f, yb + r0 + r).cst != CST_NONE;
        }
        float cen[3][3][RY][2];
#pragma unroll
        for (int t = 0; t < 3; ++t)
#pragma unroll
            for (int f = 0; f < 3; ++f)
#pragma unroll
                for (int r = 0; r < RY; ++r) cen[t][f][r][0] = cen[t][f][r][1] = 0.f;
        // output rows: their addresses on plane z0, advanced a plane per
        // update, and whether this lane stores there
        RD_GLOBAL T* po[3][RY];
        bool rowst[RY];
        // stochastic rounding: the counter of the lane pair's cells on plane
        // z0 (dense index / 4, modulo 2^32), the step and the key of species 0
        unsigned pc[RY];
        SrState sr{};
        sr.dpc = unsigned((unsigned long long)unsigned(a.nx) * unsigned(a.ny) >> 2);
        sr.have = false;
        if constexpr (ST == STORE_SR) {
            sr.n = unsigned(cload_ptr<StepClock>(a.clk_in)->n);
            sr.key = a.sr_key + unsigned(a.sp0);
        }
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int y = yb + r0 + r;
            rowst[r] = y < a.ny && (!XF || xl < a.nx);
#pragma unroll
            for (int s = 0; s < 3; ++s)
                po[s][r] = gstore_ptr<T>(a.out[s]) + ((long long)z0 * a.plane + (long long)y * a.pitch + xl);
            pc[r] = unsigned((((unsigned long long)unsigned(z0) * unsigned(a.ny) + unsigned(y)) * unsigned(a.nx) +
                              unsigned(xl)) >> 2);
        }
        // planes q-1 .. q+1 take no z rule unless q <= 1 or q >= nz - 2
        const int q_hi = a.nz - 2;
        int sc = DC - 1;                  // C slot of plane q (plane z0-2 is slot 0)
        int sab = DAB - 2;                // A/B slot of plane q (plane z0-1 is slot 0)
        // one plane: FX false compiles only the rule-free forms (planes two or
        // more inside the z faces of a wave with no fixed rows)
        auto plane = [&](int q, auto fx) __attribute__((always_inline)) {
            constexpr bool FX = decltype(fx)::value;
            lds_done();
            ring_barrier();
            const int sc1 = sc + 1 == DC ? 0 : sc + 1, sab1 = sab + 1 == DAB ? 0 : sab + 1;
            // centre rows of plane q+1
            if (q >= z0 - 2) {
                if (FX && (wfix || q <= -1 || q >= q_hi)) centre<true>(r0, q + 1, cslot(sc1), abslot(sab1), cen[2]);
                else centre<false>(r0, q + 1, cslot(sc1), abslot(sab1), cen[2]);
            }
            // update plane q
            if (q >= z0) {
                const RD_LDS T* PC = cslot(sc);
                const RD_LDS T* PAB = abslot(sab);
                if (FX && (wfix || q <= 1 || q >= q_hi))
                    update<true, CD, ST>(r0, q, PC, PAB, cen[0], cen[1], cen[2], po, rowst, pc, sr);
                else
                    update<false, CD, ST>(r0, q, PC, PAB, cen[0], cen[1], cen[2], po, rowst, pc, sr);
                sr.have = !sr.have;
#pragma unroll
                for (int r = 0; r < RY; ++r) {
#pragma unroll
                    for (int s = 0; s < 3; ++s) po[s][r] += a.plane;
                    pc[r] += sr.dpc;
                }
            }
#pragma unroll
            for (int f = 0; f < 3; ++f)
#pragma unroll
                for (int r = 0; r < RY; ++r)
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        cen[0][f][r][i] = cen[1][f][r][i];
                        cen[1][f][r][i] = cen[2][f][r][i];
                    }
            sc = sc1;
            sab = sab1;
        };
        // planes 2 .. nz-3 take the rule-free forms unless the wave has fixed rows
        const int qa = z0 - 3, qb = wfix ? qa : max(qa, min(z1, 2)), qc = wfix ? qa : max(qb, min(z1, q_hi));
        for (int q = qa; q < qb; ++q) plane(q, std::true_type{});
        for (int q = qb; q < qc; ++q) plane(q, std::false_type{});
        for (int q = qc; q < z1; ++q) plane(q, std::true_type{});
    }

    __device__ __forceinline__ void run(int cw, int z0, int z1) const {
        if (cw >= WU) {
            run_mu(cw - WU, z0, z1);
            return;
        }
        const bool cd = a.kx[2] != 0.f || a.ky[2] != 0.f || a.kz[2] != 0.f || a.p[5] != 0.f;
        const bool plain = a.rk_w == 0.f && !a.sr;
        // lane pairs start at multiples of four in the dense index when the
        // rows are a multiple of four long (x tiles start at multiples of 128)
        const bool srp = std::is_same_v<S, StBF16> && a.rk_w == 0.f && a.sr && (a.nx & 3) == 0;
        if (cd) {
            if (plain) run_update<true, STORE_PLAIN>(cw, z0, z1);
            else if (srp) run_sr<true>(cw, z0, z1);
            else run_update<true, STORE_ANY>(cw, z0, z1);
        } else {
            if (plain) run_update<false, STORE_PLAIN>(cw, z0, z1);
            else if (srp) run_sr<false>(cw, z0, z1);
            else run_update<false, STORE_ANY>(cw, z0, z1);
        }
    }

    template <bool CD>
    __device__ __forceinline__ void run_sr(int cw, int z0, int z1) const {
        if constexpr (std::is_same_v<S, StBF16>) run_update<CD, STORE_SR>(cw, z0, z1);
    }
};

template <class S, int BY, int WU, int WM, int DC>
__global__ __launch_bounds__(64 * (1 + WU + WM)) void fch_kernel(const StepArgs* __restrict__ pa) {
    using F = Fch<S, BY, DC>;
    static_assert(BY % WU == 0 && 2 * F::MROWS <= 64, "rows per wave");
    __shared__ __attribute__((aligned(16))) float ring_c[DC * F::SLOTC_W];
    __shared__ __attribute__((aligned(16))) float ring_ab[F::DAB * F::SLOTAB_W];
    __shared__ __attribute__((aligned(16))) float mring[4 * F::MSLOT];
    const StepArgs& a = *pa;
    tick_clock<FrontCH>(a, (blockIdx.x | threadIdx.x) == 0);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const TileXYZ tc = tile_coords(a, xcd_tile(blockIdx.x, gridDim.x));
    const int x0 = tc.x * F::TX;
    const int yb = tc.y * BY;
    const int z0 = tc.z * a.cz;
    const int z1 = min(z0 + a.cz, a.nz);
    RD_LDS float* rc = (RD_LDS float*)&ring_c[0];
    RD_LDS float* rab = (RD_LDS float*)&ring_ab[0];
    RD_LDS float* mb = (RD_LDS float*)&mring[0];
    if (w == 0) {
        fch_producer<S, BY, DC>(a, rc, rab, x0, yb, z0, z1);
    } else if (x0 == 0 || x0 + F::TX >= a.nx) {
        FchConsumer<S, BY, WU, WM, DC, true>(a, rc, rab, mb, x0, yb).run(w - 1, z0, z1);
    } else {
        FchConsumer<S, BY, WU, WM, DC, false>(a, rc, rab, mb, x0, yb).run(w - 1, z0, z1);
    }
}

}  // namespace rdk
