// rd_tring.hpp -- the tiled LDS ring: a z march over 128-cell x tiles of a
// block of rows, every field of the model streamed into LDS.
//
// The single-step LDS ring (rd_device.hpp, lds_kernel) keeps whole rows in
// LDS, so a model of several fields on rows of 512 cells fits only a few
// rows and one workgroup per CU.  Here a workgroup owns an x tile of 128
// cells (two per lane), rows [yb, yb+BY) and a z range [z0, z1); its ring
// holds, per plane, the tile plus one 16-byte unit on each side (the x halo)
// of BY+2 rows (one halo row each side) of every field, so two or three
// workgroups share a CU.
//
// One producer wave streams the planes into a ring of DR slots with
// direct-to-LDS loads.  Per plane q, after one barrier, each of WC computing
// waves (BY/WC rows each) updates its rows of plane q from the y-neighbour
// rows and x-halo cells of plane q that it read in the previous iteration
// and the centre rows of planes q-1, q, q+1 (registers), and reads the rows
// of plane q+1 and the centre rows of plane q+2: the LDS reads of one
// iteration are in flight during the arithmetic of the other.
//
// The cell arithmetic is the model's own cell function, as in every plan
// (so the values are bitwise those of the direct kernel); x neighbours come
// from the neighbouring lane (DPP) and the halo, y from the ring, z from
// registers.  Face rules: rows and planes beyond a face are loaded from the
// mirrored or wrapped row/plane; at the grid's x faces the producer writes
// the ring cells left of x = 0 and right of x = nx-1; fixed values and held
// faces are applied by the computing waves (a FIX variant, only where a row
// or plane of the wave is fixed, which applies the x face rules again from
// registers).
#pragma once

#include "rd_tring_cfg.hpp"

namespace rdk {

template <class M, class S, int BY, int DR>
struct Tr {
    using T = typename S::T;
    static constexpr int NF = M::NF;
    static constexpr int ES = int(sizeof(T));
    static constexpr int TX = kTrTile;             // cells of a row per workgroup
    static constexpr int HX = 16 / ES;             // halo cells per side: one 16-byte unit
    static constexpr int RW = TX + 2 * HX;         // cells per ring row: x0-HX .. x0+TX+HX-1
    static constexpr int NU = RW / HX;             // 16-byte units per ring row
    static constexpr int RR = BY + 2;              // ring rows per field: grid rows yb-1 .. yb+BY
    static constexpr int SLOT = NF * RR * RW;      // cells per slot
    static constexpr int SLOT_W = SLOT * ES / 4;   // in 4-byte words
    static_assert(NU <= 64 && RW * ES % 16 == 0 && DR >= 4, "ring layout");
};

// Every role runs iterations q = z0-3 .. tr_q_end-1, one barrier each: an
// even number, so that the computing waves can alternate two register sets
// without a tail (a last iteration past z1-1, if any, does nothing).
__host__ __device__ constexpr int tr_q_end(int z0, int z1) { return z0 - 3 + ((z1 - z0 + 4) & ~1); }

// The producer issues steps: step k loads plane z0-1+k (planes z0-1 .. z1)
// of every field into slot k mod DR.  Plane p is first read at iteration p-2
// (its centre rows), so step k must have landed before barrier z0-3+k; after
// barrier q the slot of plane q (last read at iteration q-1) is free and
// takes step q+DR+1-z0, which leaves DR-3 steps in flight.
//
// With NP producer waves, wave P loads (and patches) the ring rows
// i = f*RR + j (field f, row j) with i mod NP = P.  A wave counts its own
// loads only and can wait on at most 63 of them, so a step of many rows
// (16-row tiles of two fields: 36 loads) keeps more steps in flight when its
// rows are shared between two waves.
template <class M, class S, int BY, int DR, int NP = 1, int P = 0>
__device__ __forceinline__ void tr_producer(const StepArgs& a, RD_LDS float* ring, int x0, int yb, int z0,
                                            int z1) {
#ifndef __HIP_DEVICE_COMPILE__
    (void)a, (void)ring, (void)x0, (void)yb, (void)z0, (void)z1;
#else
    using R = Tr<M, S, BY, DR>;
    using T = typename R::T;
    constexpr int NF = R::NF;
    const int lane = threadIdx.x & 63;
    // this lane's 16-byte unit of a ring row: the tile and its halo units;
    // at the grid's x faces a halo unit is loaded only for a periodic axis
    // (the unit holding cell nx-1 on the left, cells 0 .. HX-1 on the right),
    // else the face rule supplies the value
    int col[NF];
    bool act[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const bool per = a.bck[f][0] == BC_PERIODIC;
        col[f] = x0 - R::HX + lane * R::HX;
        act[f] = lane < R::NU;
        if (lane == 0 && x0 == 0) {
            col[f] = (a.nx - 1) / R::HX * R::HX;
            act[f] = per;
        }
        if (lane == R::NU - 1 && x0 + R::TX >= a.nx) {
            col[f] = 0;
            act[f] = per;
        }
    }
    // byte offset within a plane of this lane's unit of every ring row, the
    // rows resolved by the y face rules (fixed values are applied by the
    // computing waves)
    unsigned off[NF][R::RR];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int j = 0; j < R::RR; ++j) {
            const int gy = resolve_axis(yb - 1 + j, a.ny, a.bck[f][2], a.bck[f][3], a.bcv[f][2], a.bcv[f][3]).idx;
            off[f][j] = unsigned(((long long)gy * a.pitch + col[f]) * R::ES);
        }
    const long long pbytes = a.plane * R::ES;
    const int last = z1 + 1 - z0;                  // the last step that loads
    auto plane_of = [&](int f, int p) __attribute__((always_inline)) {
        const int pz = unsigned(p) < unsigned(a.nz)
                           ? p
                           : resolve_axis(p, a.nz, a.bck[f][4], a.bck[f][5], a.bcv[f][4], a.bcv[f][5]).idx;
        return (const RD_GLOBAL char*)a.in[f] + pz * pbytes;
    };
    int slot = 0;                                  // steps are issued in order
    auto issue = [&](int k) __attribute__((always_inline)) {
        if (k <= last) {
            RD_LDS T* sl = (RD_LDS T*)(ring + slot * R::SLOT_W);
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const RD_GLOBAL char* base = plane_of(f, z0 - 1 + k);
#pragma unroll
                for (int j = 0; j < R::RR; ++j)
                    if ((f * R::RR + j) % NP == P && act[f])
                        __builtin_amdgcn_global_load_lds((const RD_GLOBAL void*)(base + off[f][j]),
                                                         (RD_LDS void*)(sl + (f * R::RR + j) * R::RW), 16, 0, 0);
            }
        }
        slot = slot + 1 == DR ? 0 : slot + 1;
    };
    // At the grid's x faces the ring cell left of x = 0 and the one right of
    // x = nx-1 (in the tile, or the halo unit) take the face rule's value once
    // a step has landed, so the computing waves read every x neighbour from
    // the ring.  Lane j patches ring row j of each field.
    const bool lface = x0 == 0, rface = x0 + R::TX >= a.nx;
    const int pr = a.nx - x0 + R::HX;              // ring cell of x = nx
    int patched = -1, pslot = 0;                   // last patched step, slot of the next
    auto patch = [&](int k) __attribute__((always_inline)) {
        // one field at a time, so that its face rule is a scalar
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            if (k > last || lane >= R::RR || (f * R::RR + lane) % NP != P) continue;
            RD_LDS T* r = (RD_LDS T*)(ring + pslot * R::SLOT_W) + (f * R::RR + lane) * R::RW;
            if (lface) {
                const int kl = a.bck[f][0];
                const T v = kl == BC_PERIODIC ? lds_peek(r + (a.nx - 1) % R::HX)
                            : kl == BC_MIRROR ? lds_peek(r + R::HX) : S::down(a.bcv[f][0]);
                lds_poke(r + R::HX - 1, v);
            }
            if (rface) {
                const int kr = a.bck[f][1];
                const T v = kr == BC_PERIODIC ? lds_peek(r + R::HX + R::TX)
                            : kr == BC_MIRROR ? lds_peek(r + pr - 1) : S::down(a.bcv[f][1]);
                lds_poke(r + pr, v);
            }
        }
        pslot = pslot + 1 == DR ? 0 : pslot + 1;
    };
    for (int k = 0; k < DR - 2; ++k) issue(k);
    constexpr int PER = (NF * R::RR - P + NP - 1) / NP;   // this wave's loads per step
    constexpr int STEADY = (DR - 3) * PER < 63 ? (DR - 3) * PER : 63;
    for (int q = z0 - 3; q < tr_q_end(z0, z1); ++q) {
        // step q+3-z0 complete: the steps issued after it may stay in flight
        const int need = q + 3 - z0;
        if (need + DR - 3 <= last) {
            vm_wait_imm<STEADY>();
        } else {
            int after = 0;
#pragma unroll
            for (int j = 1; j <= DR - 3; ++j) after += need + j <= last ? PER : 0;
            vm_wait_count<0, 63>(min(after, 63));
        }
        if (lface || rface) {
            while (patched < need) patch(++patched);
            lds_done();
        }
        ring_barrier();
        issue(q + DR + 1 - z0);
    }
#endif
}

// A computing wave: RY = BY / WC output rows, two cells per lane.  PK
// (rows of at most 64 cells): lanes 0-31 and 32-63 take two rows at once, so
// a wave makes RY/2 passes over its rows instead of RY.
template <class M, class S, int BY, int WC, int DR, bool PK = false>
struct TrConsumer {
    using R = Tr<M, S, BY, DR>;
    using T = typename R::T;
    static constexpr int NF = M::NF, NO = M::NO, RY = BY / WC;
    static constexpr int RYE = PK ? RY / 2 : RY;   // passes over the wave's rows
    static_assert(!PK || RY % 2 == 0, "packed rows come in pairs");
    static constexpr int HX = R::HX, TX = R::TX, RW = R::RW, RR = R::RR;

    const StepArgs& a;
    const CellConst k;
    const RD_LDS T* ring;
    int lane, sub, cl, x0, yb, xl;
    __device__ __forceinline__ TrConsumer(const StepArgs& a_, const RD_LDS float* ring_w, int x0_, int yb_)
        : a(a_), k(a_), ring((const RD_LDS T*)ring_w), lane(threadIdx.x & 63),
          sub(PK ? (threadIdx.x & 63) >> 5 : 0), cl(PK ? threadIdx.x & 31 : threadIdx.x & 63), x0(x0_), yb(yb_),
          xl(x0_ + 2 * (PK ? threadIdx.x & 31 : threadIdx.x & 63)) {}
    // wave row of pass r (this lane's row when packed)
    __device__ __forceinline__ int prow(int r0, int r) const { return PK ? r0 + 2 * r + sub : r0 + r; }

    __device__ __forceinline__ const RD_LDS T* slot(int s) const { return ring + s * R::SLOT; }
    static __device__ __forceinline__ const RD_LDS T* row(const RD_LDS T* P, int f, int j) {
        return P + (f * RR + j) * RW;
    }
    // this lane's two cells of a ring row, as FP32
    __device__ __forceinline__ void rd2(const RD_LDS T* r, float (&o)[2]) const {
        const RD_LDS T* q = r + HX + 2 * cl;
        if constexpr (sizeof(T) == 4) {
            typedef float v2f __attribute__((ext_vector_type(2)));
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
    // LDS cell of x0-1 (at the grid's left face the producer's patch)
    static constexpr int HL = HX - 1;
    // The producer's patch holds a fixed x-face value of field f in the
    // storage type; where that rounds it, the face is applied from registers
    // (the FIX variant) instead.
    __device__ __forceinline__ bool xface_rounded(int f) const {
        bool r = false;
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const bool at = side == 0 ? x0 == 0 : x0 + TX >= a.nx;
            const int kind = a.bck[f][side];
            const float v = a.bcv[f][side];
            r = r || (at && kind != BC_MIRROR && kind != BC_PERIODIC && S::up(S::down(v)) != v);
        }
        return r;
    }

    // x neighbours of this lane's two cells (values v; halo cells hl = x0-1,
    // hr = x0+TX); FIX: the x face rules of field f applied again at the
    // grid's faces (the values of a fixed row differ from the loaded ones)
    template <bool FIX>
    __device__ __forceinline__ void xnb(int f, const float (&v)[2], float hl, float hr, float (&xm)[2],
                                        float (&xp)[2]) const {
        float fill = hl;
        if constexpr (FIX) {
            const int kl = a.bck[f][0];
            if (x0 == 0 && kl != BC_PERIODIC) fill = kl == BC_MIRROR ? v[0] : a.bcv[f][0];
        }
        xm[0] = lane_from_left(v[1], fill);
        xm[1] = v[0];
        xp[0] = v[1];
        xp[1] = lane_from_right(v[0], hr);
        if constexpr (PK) {
            // the lane groups' own ends: the neighbour lane holds the other row
            // (lane 31's right neighbour matters only for rows of 64 cells,
            // where hr is x = 64)
            if (cl == 0) xm[0] = fill;
            if (cl == 31) xp[1] = hr;
        }
        if constexpr (FIX) {
            if (x0 + TX >= a.nx) {
                const int kr = a.bck[f][1];
                const float fv = a.bcv[f][1];
                if (xl == a.nx - 1) xp[0] = kr == BC_MIRROR ? v[0] : kr == BC_PERIODIC ? hr : fv;
                if (xl + 1 == a.nx - 1) xp[1] = kr == BC_MIRROR ? v[1] : kr == BC_PERIODIC ? hr : fv;
            }
        }
    }

    // centre rows of the wave's output rows (slot P) as read, and their rules
    // applied once they are in
    __device__ __forceinline__ void centre_read(int r0, const RD_LDS T* P, float (&c)[NF][RYE][2]) const {
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int r = 0; r < RYE; ++r) rd2(row(P, f, prow(r0, r) + 1), c[f][r]);
    }
    __device__ __forceinline__ void centre_fix(int r0, int p, float (&c)[NF][RYE][2]) const {
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int r = 0; r < RYE; ++r) fix_row<2>(a, f, zsrc(f, p), ysrc(f, yb + prow(r0, r)), xl, c[f][r]);
    }

    // the y neighbour rows and x halo cells of the output rows of one plane
    struct RowsIn {
        float ym[NF][RYE][2], yp[NF][RYE][2], hl[NF][RYE], hr[NF][RYE];
    };
    __device__ __forceinline__ void rows_read(int r0, const RD_LDS T* P, RowsIn& in) const {
        const int hlo = HL;
#pragma unroll
        for (int r = 0; r < RYE; ++r)
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const int j = prow(r0, r) + 1;
                const RD_LDS T* rc = row(P, f, j);
                rd2(row(P, f, j - 1), in.ym[f][r]);
                rd2(row(P, f, j + 1), in.yp[f][r]);
                in.hl[f][r] = rd1(rc, hlo);
                // the cell right of the lane group: x0+TX, or for packed rows x = nx,
                // which the producer's patch holds (the wrapped value on a
                // periodic axis, as the halo unit at x0+TX does unpacked)
                in.hr[f][r] = rd1(rc, HX + (PK ? a.nx : TX));
            }
    }

    // the outputs of plane z on rows r0 ..: neighbours from `in` (plane z) and
    // the centre rows of z-1, z, z+1.  PLAIN: no Runge-Kutta combination and
    // no stochastic rounding in the stores.
    template <bool FIX, bool PLAIN>
    __device__ __forceinline__ void update(int r0, int z, RowsIn in, const float (&cm)[NF][RYE][2],
                                           const float (&c0)[NF][RYE][2], const float (&cp)[NF][RYE][2],
                                           RD_GLOBAL T* const (&po)[NO][RYE], const bool (&rowst)[RYE]) const {
        const float wind = plane_wind<M>(a, z);
#pragma unroll
        for (int r = 0; r < RYE; ++r) {
            const int y = yb + prow(r0, r);
            Nb n[2][NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                if constexpr (FIX) {
                    const Src pz = zsrc(f, z), y0 = ysrc(f, y);
                    fix_row<2>(a, f, pz, ysrc(f, y - 1), xl, in.ym[f][r]);
                    fix_row<2>(a, f, pz, ysrc(f, y + 1), xl, in.yp[f][r]);
                    fix1(a, f, pz, y0, x0 == 0 ? a.nx - 1 : x0 - 1, in.hl[f][r]);
                    fix1(a, f, pz, y0, x0 + (PK ? a.nx : TX), in.hr[f][r]);
                }
                float xm[2], xp[2];
                xnb<FIX>(f, c0[f][r], in.hl[f][r], in.hr[f][r], xm, xp);
#pragma unroll
                for (int i = 0; i < 2; ++i)
                    n[i][f] = Nb{c0[f][r][i], xm[i], xp[i], in.ym[f][r][i], in.yp[f][r][i], cm[f][r][i], cp[f][r][i]};
            }
            // the row's sources (a row past the grid's last reads none: its
            // entries would lie beyond the table)
            int s0 = 0, s1 = 0;
            if constexpr (M::SOURCES) {
                if (y < a.ny) {
                    const int rr = z * a.ny + y;
                    s0 = cload_ptr<int>(a.src_row)[rr];
                    s1 = cload_ptr<int>(a.src_row)[rr + 1];
                }
            }
            float o[NO][2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                Emission<NO> em{};
                if constexpr (M::SOURCES) em = cell_sources<NO>(a, xl + i, s0, s1);
                float oi[NO];
                M::cell(k, n[i], wind, em.any, em.e, oi);
#pragma unroll
                for (int s = 0; s < NO; ++s) o[s][i] = FIX ? held_out(a, s, xl + i, y, z, oi[s]) : oi[s];
            }
            if (rowst[r]) {
                if constexpr (PLAIN) {
#pragma unroll
                    for (int s = 0; s < NO; ++s) store_vec_at<S, 2>(po[s][r], o[s]);
                } else {
#pragma unroll
                    for (int s = 0; s < NO; ++s) store_field<S, 2>(a, s, xl, y, z, o[s]);
                }
            }
        }
    }

    // one computing wave (index cw) over the z range: planes z0 .. z1-1
    template <bool PLAIN>
    __device__ __forceinline__ void run(int cw, int z0, int z1) const {
        const int r0 = cw * RY;
        bool wfix = false;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            wfix = wfix || (a.held[f] & 3) != 0 || xface_rounded(f);
#pragma unroll
            for (int r = -1; r <= RY; ++r) wfix = wfix || ysrc(f, yb + r0 + r).cst != CST_NONE;
        }
        // centre rows of planes q-1, q, q+1 and (read in iteration q) q+2
        float cen[4][NF][RYE][2];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int f = 0; f < NF; ++f)
#pragma unroll
                for (int r = 0; r < RYE; ++r) cen[t][f][r][0] = cen[t][f][r][1] = 0.f;
        // output rows: their addresses on plane z0, advanced a plane per
        // update, and whether this lane stores there
        RD_GLOBAL T* po[NO][RYE];
        bool rowst[RYE];
#pragma unroll
        for (int r = 0; r < RYE; ++r) {
            const int y = yb + prow(r0, r);
            rowst[r] = y < a.ny && xl < a.nx;
#pragma unroll
            for (int s = 0; s < NO; ++s)
                po[s][r] = gstore_ptr<T>(a.out[s]) + ((long long)z0 * a.plane + (long long)y * a.pitch + xl);
        }
        // planes q-1 .. q+1 take no z rule unless q <= 1 or q >= nz - 2
        const int q_hi = a.nz - 2;
        int s1 = DR - 1;                  // slot of plane q+1 (plane z0-1 is slot 0)
        auto body = [&](int q, RowsIn& rd, const RowsIn& cur) __attribute__((always_inline)) {
            lds_done();
            ring_barrier();
            const int s2 = s1 + 1 == DR ? 0 : s1 + 1;    // slot of plane q+2
            if (q + 1 >= z0 && q + 1 < z1) rows_read(r0, slot(s1), rd);
            const bool cen_next = q + 2 >= z0 - 1 && q + 2 <= z1;
            if (cen_next) centre_read(r0, slot(s2), cen[3]);
            __builtin_amdgcn_sched_barrier(0);
            if (q >= z0 && q < z1) {
                if (wfix || q <= 1 || q >= q_hi)
                    update<true, PLAIN>(r0, q, cur, cen[0], cen[1], cen[2], po, rowst);
                else
                    update<false, PLAIN>(r0, q, cur, cen[0], cen[1], cen[2], po, rowst);
#pragma unroll
                for (int s = 0; s < NO; ++s)
#pragma unroll
                    for (int r = 0; r < RYE; ++r) po[s][r] += a.plane;
            }
            if (cen_next && (wfix || q + 2 <= 0 || q + 2 >= a.nz - 1)) centre_fix(r0, q + 2, cen[3]);
#pragma unroll
            for (int f = 0; f < NF; ++f)
#pragma unroll
                for (int r = 0; r < RYE; ++r)
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        cen[0][f][r][i] = cen[1][f][r][i];
                        cen[1][f][r][i] = cen[2][f][r][i];
                        cen[2][f][r][i] = cen[3][f][r][i];
                    }
            s1 = s2;
        };
        // two sets of rows trade roles every iteration (no copies)
        RowsIn ra, rb;
        for (int q = z0 - 3; q < tr_q_end(z0, z1); q += 2) {
            body(q, ra, rb);
            body(q + 1, rb, ra);
        }
    }
};

// One workgroup's march over its tile (waves 0 .. NP-1 load, the others
// compute).
// PKOK: rows of at most 64 cells (pk) take the packed computing waves.
template <class M, class S, int BY, int WC, int DR, bool PLAIN, int NP = 1, bool PKOK = false>
__device__ __forceinline__ void tr_run(const StepArgs& a, RD_LDS float* rg, int w, int x0, int yb, int z0, int z1,
                                       bool pk = false) {
    static_assert(NP == 1 || NP == 2, "one or two producer waves");
    if (w == 0) tr_producer<M, S, BY, DR, NP, 0>(a, rg, x0, yb, z0, z1);
    else if (NP == 2 && w == 1) tr_producer<M, S, BY, DR, NP, NP - 1>(a, rg, x0, yb, z0, z1);
    else if (PKOK && pk) TrConsumer<M, S, BY, WC, DR, PKOK>(a, rg, x0, yb).template run<PLAIN>(w - NP, z0, z1);
    else TrConsumer<M, S, BY, WC, DR>(a, rg, x0, yb).template run<PLAIN>(w - NP, z0, z1);
}

// PLAIN: the launch has no Runge-Kutta combination and no stochastic
// rounding, so only that store is compiled into it.  Waves: tr_np loading
// waves, then WC computing waves.
template <class M, class S, int BY, int WC, int DR, bool PLAIN>
__global__ __launch_bounds__(64 * (tr_np(M::NF, BY, DR) + WC)) void tr_kernel(const StepArgs* __restrict__ pa) {
    using R = Tr<M, S, BY, DR>;
    static_assert(BY % WC == 0, "rows per wave");
    __shared__ __attribute__((aligned(16))) float ring[DR * R::SLOT_W];
    const StepArgs& a = *pa;
    tick_clock<M>(a, (blockIdx.x | threadIdx.x) == 0);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const TileXYZ tc = tile_coords(a, xcd_tile(blockIdx.x, gridDim.x));
    const int z0 = tc.z * a.cz;
    tr_run<M, S, BY, WC, DR, PLAIN, tr_np(M::NF, BY, DR)>(a, (RD_LDS float*)&ring[0], w, tc.x * R::TX,
                                                         tc.y * BY, z0, min(z0 + a.cz, a.nz));
}

// The batched form (served grids of diffusion or the Brusselator, forward
// Euler, round-to-nearest stores): a persistent launch walks the batch's
// (grid, tile) items, each item a tile of 128-cell rows marching a z chunk
// of its grid.  The host writes the table (rd_device.hpp, BatchEntry) with
// each grid's arguments tiled for this kernel, largest items first.
// Workgroups claim items from a ticket counter, so the step ends when the
// last item does however unequal the items are; the last workgroup to finish
// puts both counters back to zero for the next launch.
template <class S, int BY, int WC, int DR, int NP>
__global__ __launch_bounds__(64 * (NP + WC)) void batched_tr_kernel(int* __restrict__ meta,
                                                                    const BatchEntry* __restrict__ ents, int step) {
    // one ring serves both models (sized for the Brusselator's two fields)
    using RB = Tr<Brusselator, S, BY, DR>;
    static_assert(Tr<Diffusion<1>, S, BY, DR>::SLOT_W <= RB::SLOT_W, "batch ring");
    __shared__ __attribute__((aligned(16))) float ring[DR * RB::SLOT_W];
    __shared__ int claimed;
    const int ng = meta[0];
    const int total = meta[1];
    int* ticket = meta + 2;
    int* finished = meta + 3;
    const int* first = meta + 4;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    RD_LDS float* rg = (RD_LDS float*)&ring[0];
    for (;;) {
        if (threadIdx.x == 0) claimed = atomicAdd(ticket, 1);
        __syncthreads();
        const int item = claimed;
        __syncthreads();                         // every wave has read it
        if (item >= total) break;
        int lo = 0, hi = ng - 1;                 // last grid with first_item <= item
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (first[mid] <= item) lo = mid; else hi = mid - 1;
        }
        const BatchEntry& en = ents[lo];
        if (step >= en.steps_left) continue;     // this grid already finished
        const StepArgs& a = en.args[(en.parity + step) & 1];
        const TileXYZ tc = tile_coords(a, item - first[lo]);
        const int z0 = tc.z * a.cz, z1 = min(z0 + a.cz, a.nz);
        // rows of at most 64 cells: two rows per lane group pass (two cells per lane)
        constexpr bool PKOK = (BY / WC) % 2 == 0;
        const bool pk = a.nx <= 64;
        if (en.model == 1)
            tr_run<Brusselator, S, BY, WC, DR, true, NP, PKOK>(a, rg, w, tc.x * kTrTile, tc.y * BY, z0, z1, pk);
        else
            tr_run<Diffusion<1>, S, BY, WC, DR, true, NP, PKOK>(a, rg, w, tc.x * kTrTile, tc.y * BY, z0, z1, pk);
        __syncthreads();                         // the next item refills the ring
    }
    if (threadIdx.x == 0) {
        __threadfence();                         // this workgroup's claims come first
        if (atomicAdd(finished, 1) == int(gridDim.x) - 1) {
            __threadfence();                     // after every other workgroup's claims
            atomicExch(ticket, 0);
            atomicExch(finished, 0);
        }
    }
}

}  // namespace rdk
