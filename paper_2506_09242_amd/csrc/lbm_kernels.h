// lbm_kernels.h -- the fused collide-and-stream kernel and its helpers.
//
// Included by one translation unit per (Q, precision); each instantiates the
// launchers declared in lbm_internal.h.
//
// In-place streaming: the AA pattern (named in Sec. 2.3 of the paper as the
// single-array, thread-safe alternative to the two-population scheme).
// With h_i(x) the population of direction i at node x stored in slot i:
//   even step  : read slot i at x; collide; write h*_i to slot opp(i) at x.
//   odd step   : read h_i(x) from slot opp(i) at x - c_i; collide; write h*_i
//                to slot i at x + c_i.
// After an even step the array holds the next state "in reverse"; after the
// odd step it is back in natural layout.  Each (node, slot) is read and
// written by exactly one thread per step, so the update is race-free.
// Half-way bounce-back (Sec. 3 intro, after Ladd) closes the loop next to a
// non-fluid node y = x + c_i: the post-collision h*_i returns to node x as
// direction opp(i), minus 6 w_i rho0 (c_i . u_wall) for a moving wall; in
// the even step that value already sits in slot opp(i) at x (so the wall
// term is applied there), in the odd step it is written to slot opp(i) at x,
// and the odd step's read of direction i from a wall neighbour x - c_i
// takes slot i at x instead.
//
// Node update (Sec. 2.3 push-pull scheme): the Q populations of a node are
// pulled into registers, the tag selects the collision model among the
// compiled model set (BGK, TRT, BGK with Smagorinsky or the learned eddy
// viscosity, regularized BGK, regularized open boundaries), and the results
// are pushed back (slot addresses from pop_base / slot_off).  Populations are
// stored shifted, h_i = f_i - w_i rho0 (Sec. 3 intro, Skordos' offset
// stripping), which the collision is written for directly:
//   drho = sum h_i, rho = rho0 + drho, j = sum c_i h_i, u = (j + F/2) / rho
//   heq_i = w_i (drho + rho (3 c.u + 9/2 (c.u)^2 - 3/2 u.u))
// and the collision works on pairs (i, opp(i)) split into even and odd parts
// (TRT; BGK is the case omega- = omega+), with the Guo forcing term split
// the same way.
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_device.h"
#include "lbm_internal.h"
#include "lbm_mlp_device.h"

namespace lbmd {

// Per-node neighbour mask layout.  Fluid node: bits 1..26 wall bits (bit i
// set when node x + c_i is not fluid), bit 27 set when a neighbour is a moving
// wall, bits 28..31 the node's own fluid tag.  Non-fluid node (tag bits 0):
// zero, or a filler (see the step kernel) with bit 0 set and bit i set when
// node x + (0, c_iy, c_iz) is not fluid.
constexpr uint32_t kMaskWalls = (1u << 27) - 1u;
constexpr int kMaskMovingBit = 27;
constexpr int kMaskTagShift = 28;

__device__ __forceinline__ int wrap_idx(int v, int n) { return v < 0 ? v + n : (v >= n ? v % n : v); }

// FP64 reduction terms of one node's loaded (time-t) populations, added to red.
template <int Q, typename C>
__device__ __forceinline__ void node_reduce(const C (&h)[Q], bool live, const StepParams &p, double (&red)[NRED]) {
    double dr = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    sfor<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        using Vi = V<Q, i>;
        const double v = (double)h[i];
        dr += v;
        if constexpr (Vi::x != 0) jx += Vi::x * v;
        if constexpr (Vi::y != 0) jy += Vi::y * v;
        if constexpr (Vi::z != 0) jz += Vi::z * v;
    });
    const double rho = p.rho0 + dr;
    const double px = jx + 0.5 * p.force[0], py = jy + 0.5 * p.force[1], pz = jz + 0.5 * p.force[2];
    const double ux = px / rho, uy = py / rho, uz = pz / rho;
    const double uu = ux * ux + uy * uy + uz * uz;
    const bool ok = isfinite(rho) && isfinite(uu);
    const bool use = live && ok;
    red[0] += use ? dr : 0.0;
    red[1] += use ? px : 0.0;
    red[2] += use ? py : 0.0;
    red[3] += use ? pz : 0.0;
    red[4] += use ? ux : 0.0;
    red[5] += use ? uy : 0.0;
    red[6] += use ? uz : 0.0;
    red[7] += use ? 0.5 * uu : 0.0;
    red[8] += use ? 0.5 * rho * uu : 0.0;
    red[9] += (live && !ok) ? 1.0 : 0.0;
}

// Regularized open boundary on an x plane (the conditions of Latt et al. 2008
// the paper uses for the Berea runs, Sec. 3.3), shifted form: f_i = h_i + w_i rho0.
// On the x = 0 plane the populations with c_x = +1 come from outside, on
// x = nx-1 those with c_x = -1.  Mass and x-momentum over the known populations
// give, with s = -1 on x = 0 and s = +1 on x = nx-1,
//   rho (1 + s u_x) = sum_{c_x=0} f + 2 sum_{c_x=s} f = s0 + 2 s_s + rho0 = K
// (the weights of c_x = 0 plus twice those of c_x = s sum to 1): a velocity
// boundary (u imposed) has rho = K / (1 + s u_x), a pressure boundary (rho
// imposed, u_y = u_z = 0) has u_x = s (K / rho - 1).  Each unknown population
// is equilibrium plus its opposite's non-equilibrium part; the node is then
// regularized (Hermite projection of its momentum flux) and relaxed with omega.
// No body force on these nodes.
template <int Q, typename C>
__device__ __forceinline__ void open_boundary(const C (&h)[Q], int tag, const StepParams &p, C (&hs)[Q]) {
    const bool low = tag == LBM_TAG_VEL_IN || tag == LBM_TAG_PRES_IN;  // the x = 0 plane
    const bool vel = tag == LBM_TAG_VEL_IN || tag == LBM_TAG_VEL_OUT;  // velocity imposed
    C s0 = C(0), sp = C(0), sm = C(0);
    sfor<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        using Vi = V<Q, i>;
        if constexpr (Vi::x == 0) s0 += h[i];
        if constexpr (Vi::x > 0) sp += h[i];
        if constexpr (Vi::x < 0) sm += h[i];
    });
    const C rho0 = (C)p.rho0;
    const C sg = low ? C(-1) : C(1);
    const C K = s0 + C(2) * (low ? sm : sp) + rho0;
    C rb, ux, uy, uz;
    if (vel) {
        ux = (C)p.bc_u[0];
        uy = (C)p.bc_u[1];
        uz = (C)p.bc_u[2];
        rb = K / (C(1) + sg * ux);
    } else {
        rb = (C)p.bc_rho[low ? 0 : 1];
        ux = sg * (K / rb - C(1));
        uy = C(0);
        uz = C(0);
    }
    const C drb = rb - rho0;
    const C uu = ux * ux + uy * uy + uz * uz;
    C he[Q];
    sfor<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        using Vi = V<Q, i>;
        C cu = C(0);
        if constexpr (Vi::x != 0) cu += C(Vi::x) * ux;
        if constexpr (Vi::y != 0) cu += C(Vi::y) * uy;
        if constexpr (Vi::z != 0) cu += C(Vi::z) * uz;
        he[i] = C(Vi::w) * (drb + rb * (C(3) * cu + C(4.5) * cu * cu - C(1.5) * uu));
    });
    // non-equilibrium part of the completed node; an unknown population takes
    // its opposite's
    C pxx = C(0), pyy = C(0), pzz = C(0), pxy = C(0), pxz = C(0), pyz = C(0);
    sfor<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        using Vi = V<Q, i>;
        if constexpr (i > 0) {
            constexpr int o = Vi::opp;
            C ne = h[i] - he[i];
            if constexpr (Vi::x != 0) {
                const bool unknown = low ? (Vi::x > 0) : (Vi::x < 0);
                if (unknown) ne = h[o] - he[o];
            }
            if constexpr (Vi::x != 0) pxx += ne;
            if constexpr (Vi::y != 0) pyy += ne;
            if constexpr (Vi::z != 0) pzz += ne;
            if constexpr (Vi::x * Vi::y != 0) pxy += C(Vi::x * Vi::y) * ne;
            if constexpr (Vi::x * Vi::z != 0) pxz += C(Vi::x * Vi::z) * ne;
            if constexpr (Vi::y * Vi::z != 0) pyz += C(Vi::y * Vi::z) * ne;
        }
    });
    const C tr = (pxx + pyy + pzz) * C(1.0 / 3.0);
    const C a = (C(1) - (C)p.omega) * C(4.5);
    sfor<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        using Vi = V<Q, i>;
        C cpc = C(0);
        if constexpr (Vi::x != 0) cpc += pxx;
        if constexpr (Vi::y != 0) cpc += pyy;
        if constexpr (Vi::z != 0) cpc += pzz;
        if constexpr (Vi::x * Vi::y != 0) cpc += C(2 * Vi::x * Vi::y) * pxy;
        if constexpr (Vi::x * Vi::z != 0) cpc += C(2 * Vi::x * Vi::z) * pxz;
        if constexpr (Vi::y * Vi::z != 0) cpc += C(2 * Vi::y * Vi::z) * pyz;
        hs[i] = he[i] + a * C(Vi::w) * (cpc - tr);
    });
}

// Collision of one node in shifted form (pair split, Guo forcing).  Every lane
// of the wave must call it (the learned closure is evaluated wave-wide).
// Regularized and recursive-regularized update for lattices whose fluid nodes
// all use one of those two models.  Both relax to a state built from the
// moments alone (rho, u and the non-equilibrium momentum flux), so the update
// needs the populations only for the moment sums: the flux comes from the
// second moment of h minus that of the equilibrium,
//   Pi_ab = sum c_a c_b h - drho / 3 delta_ab - rho u_a u_b
// (h = f - w rho0; the second-order equilibrium's second moment is
// rho / 3 delta + rho u u on D3Q19 and D3Q27), and the post-collision pair
// (k, k + H) is feq_k + F_k / 2 + the regularized (and third-order) terms,
// with the odd parts entering with opposite signs.  The same algebra as the
// general path with omega = 1 in its relaxation, where h cancels; only the
// rounding differs.  Keeping no population live across the update frees the
// registers the general path needs.
template <int Q, typename C, int MS>
__device__ __forceinline__ void collide_regularized(const C (&h)[Q], int tag, const StepParams &p, C (&hs)[Q]) {
    constexpr int H = (Q - 1) / 2;
    constexpr bool RR = MS == MS_RR;
    C drho = C(0), jx = C(0), jy = C(0), jz = C(0);
    C sxx = C(0), syy = C(0), szz = C(0), sxy = C(0), sxz = C(0), syz = C(0);
    sfor<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        using Vi = V<Q, i>;
        drho += h[i];
        if constexpr (Vi::x == 1) jx += h[i];
        if constexpr (Vi::x == -1) jx -= h[i];
        if constexpr (Vi::y == 1) jy += h[i];
        if constexpr (Vi::y == -1) jy -= h[i];
        if constexpr (Vi::z == 1) jz += h[i];
        if constexpr (Vi::z == -1) jz -= h[i];
        if constexpr (Vi::x != 0) sxx += h[i];
        if constexpr (Vi::y != 0) syy += h[i];
        if constexpr (Vi::z != 0) szz += h[i];
        if constexpr (Vi::x * Vi::y == 1) sxy += h[i];
        if constexpr (Vi::x * Vi::y == -1) sxy -= h[i];
        if constexpr (Vi::x * Vi::z == 1) sxz += h[i];
        if constexpr (Vi::x * Vi::z == -1) sxz -= h[i];
        if constexpr (Vi::y * Vi::z == 1) syz += h[i];
        if constexpr (Vi::y * Vi::z == -1) syz -= h[i];
    });
    const C Fx = (C)p.force[0], Fy = (C)p.force[1], Fz = (C)p.force[2];
    const C rho = (C)p.rho0 + drho;
    const C inv_rho = C(1) / rho;
    const C ux = (jx + C(0.5) * Fx) * inv_rho;
    const C uy = (jy + C(0.5) * Fy) * inv_rho;
    const C uz = (jz + C(0.5) * Fz) * inv_rho;
    const C uu = ux * ux + uy * uy + uz * uz;
    const C uF = ux * Fx + uy * Fy + uz * Fz;
    const C d3 = drho * C(1.0 / 3.0);
    // Pi1 = Pi + (uF + Fu) / 2
    const C rxx = sxx - d3 - rho * ux * ux + ux * Fx;
    const C ryy = syy - d3 - rho * uy * uy + uy * Fy;
    const C rzz = szz - d3 - rho * uz * uz + uz * Fz;
    const C rxy = sxy - rho * ux * uy + C(0.5) * (ux * Fy + uy * Fx);
    const C rxz = sxz - rho * ux * uz + C(0.5) * (ux * Fz + uz * Fx);
    const C ryz = syz - rho * uy * uz + C(0.5) * (uy * Fz + uz * Fy);
    const C rtr = (rxx + ryy + rzz) * C(1.0 / 3.0);
    const bool on = tag == (RR ? LBM_TAG_RR : LBM_TAG_REG);
    const C om1 = C(1) - (C)p.omega;
    const C reg = on ? om1 * C(4.5) : C(0);
    C t1p = C(0), t1m = C(0), t2p = C(0), t2m = C(0), t3p = C(0), t3m = C(0), t7 = C(0);
    if constexpr (RR) {
        // A2 = (1 - omega) dev Pi1, A3 recursive, T = rho u u u + A3
        const C axx = om1 * (rxx - rtr), ayy = om1 * (ryy - rtr), azz = om1 * (rzz - rtr);
        const C axy = om1 * rxy, axz = om1 * rxz, ayz = om1 * ryz;
        const C txxy = rho * ux * ux * uy + C(2) * ux * axy + uy * axx;
        const C tyzz = rho * uy * uz * uz + uy * azz + C(2) * uz * ayz;
        const C txzz = rho * ux * uz * uz + ux * azz + C(2) * uz * axz;
        const C txyy = rho * ux * uy * uy + ux * ayy + C(2) * uy * axy;
        const C tyyz = rho * uy * uy * uz + C(2) * uy * ayz + uz * ayy;
        const C txxz = rho * ux * ux * uz + C(2) * ux * axz + uz * axx;
        constexpr double np_ = Q == 19 ? 27.0 / 2.0 : 27.0 / 4.0;  // 1 / norm of a sum
        constexpr double nm_ = Q == 19 ? 27.0 / 6.0 : 27.0 / 4.0;  // 1 / norm of a difference
        const C g = on ? C(1) : C(0);
        t1p = g * (txxy + tyzz) * C(np_);
        t1m = g * (txxy - tyzz) * C(nm_);
        t2p = g * (txzz + txyy) * C(np_);
        t2m = g * (txzz - txyy) * C(nm_);
        t3p = g * (tyyz + txxz) * C(np_);
        t3m = g * (tyyz - txxz) * C(nm_);
        if constexpr (Q == 27) t7 = g * (rho * ux * uy * uz + ux * ayz + uy * axz + uz * axy) * C(27.0);
    }

    // rest population: regularized keeps the trace term, recursive relaxes it with 1
    hs[0] = C(V<Q, 0>::w) * (drho - C(1.5) * rho * uu - C(1.5) * uF);
    if constexpr (!RR) hs[0] -= reg * C(V<Q, 0>::w) * rtr;
    sfor<H>([&](auto K) {
        constexpr int k = decltype(K)::value + 1;
        using Vk = V<Q, k>;
        C cu = C(0), cF = C(0), cpc = C(0);
        if constexpr (Vk::x != 0) cu += C(Vk::x) * ux, cF += C(Vk::x) * Fx, cpc += rxx;
        if constexpr (Vk::y != 0) cu += C(Vk::y) * uy, cF += C(Vk::y) * Fy, cpc += ryy;
        if constexpr (Vk::z != 0) cu += C(Vk::z) * uz, cF += C(Vk::z) * Fz, cpc += rzz;
        if constexpr (Vk::x * Vk::y != 0) cpc += C(2 * Vk::x * Vk::y) * rxy;
        if constexpr (Vk::x * Vk::z != 0) cpc += C(2 * Vk::x * Vk::z) * rxz;
        if constexpr (Vk::y * Vk::z != 0) cpc += C(2 * Vk::y * Vk::z) * ryz;
        const C ev = C(Vk::w) * (drho + rho * (C(4.5) * cu * cu - C(1.5) * uu));
        const C od = C(Vk::w) * C(3) * rho * cu;
        const C Fe = C(Vk::w) * (C(9) * cu * cF - C(3) * uF);
        const C Fo = C(Vk::w) * C(3) * cF;
        // regularized: |c|^2 -> 1 (tr Q = 0 projection); recursive: |c|^2 (deviatoric)
        const C R = reg * C(Vk::w) * (cpc - rtr * C(RR ? Vk::n2 : 1));
        C E = C(0);
        if constexpr (RR) {
            constexpr int cx = Vk::x, cy = Vk::y, cz = Vk::z;
            constexpr double p1p = cy * (cx * cx + cz * cz - 2.0 / 3.0), p1m = cy * (cx * cx - cz * cz);
            constexpr double p2p = cx * (cy * cy + cz * cz - 2.0 / 3.0), p2m = cx * (cz * cz - cy * cy);
            constexpr double p3p = cz * (cx * cx + cy * cy - 2.0 / 3.0), p3m = cz * (cy * cy - cx * cx);
            constexpr double p7 = cx * cy * cz;
            if constexpr (p1p != 0.0) E += C(p1p) * t1p;
            if constexpr (p1m != 0.0) E += C(p1m) * t1m;
            if constexpr (p2p != 0.0) E += C(p2p) * t2p;
            if constexpr (p2m != 0.0) E += C(p2m) * t2m;
            if constexpr (p3p != 0.0) E += C(p3p) * t3p;
            if constexpr (p3m != 0.0) E += C(p3m) * t3m;
            if constexpr (Q == 27 && p7 != 0.0) E += C(p7) * t7;
            E *= C(Vk::w);
        }
        const C A = ev + C(0.5) * Fe + R;
        const C B = od + C(0.5) * Fo + E;
        hs[k] = A + B;
        hs[k + H] = A - B;
    });
}

// BGK with a per-node relaxation time from the eddy-viscosity closure (tag
// BGK+MLP), from Smagorinsky (tag BGK+Smagorinsky, and the closure's
// fallback) or the plain one (tag BGK), for lattices whose fluid nodes use
// only these three models.  The non-equilibrium momentum flux comes from the
// second moment of h minus that of the second-order equilibrium (dRho/3 I +
// rho u u, exact on D3Q19 and D3Q27), and the network is evaluated before the
// equilibrium is formed, pair by pair where it is used: only the populations
// and a few moments are live across the matrix-core products.
template <int Q, typename C, int MS>
__device__ __forceinline__ void collide_closure(const C (&h)[Q], int tag, bool live, const StepParams &p,
                                                C (&hs)[Q]) {
    constexpr int H = (Q - 1) / 2;
    // moments from the pair sums and differences (the second moments see only
    // the even parts, the momentum only the odd ones)
    C drho = h[0], jx = C(0), jy = C(0), jz = C(0);
    C sxx = C(0), syy = C(0), szz = C(0), sxy = C(0), sxz = C(0), syz = C(0);
    C E[H + 1], O[H + 1];  // pair halves (h_k + h_k') / 2 and (h_k - h_k') / 2; h is not used again
    sfor<H>([&](auto K) {
        constexpr int k = decltype(K)::value + 1;
        using Vk = V<Q, k>;
        const C e = h[k] + h[k + H], o = h[k] - h[k + H];
        E[k] = C(0.5) * e;
        O[k] = C(0.5) * o;
        drho += e;
        if constexpr (Vk::x != 0) jx += C(Vk::x) * o, sxx += e;
        if constexpr (Vk::y != 0) jy += C(Vk::y) * o, syy += e;
        if constexpr (Vk::z != 0) jz += C(Vk::z) * o, szz += e;
        if constexpr (Vk::x * Vk::y != 0) sxy += C(Vk::x * Vk::y) * e;
        if constexpr (Vk::x * Vk::z != 0) sxz += C(Vk::x * Vk::z) * e;
        if constexpr (Vk::y * Vk::z != 0) syz += C(Vk::y * Vk::z) * e;
    });
    const C Fx = (C)p.force[0], Fy = (C)p.force[1], Fz = (C)p.force[2];
    const C rho = (C)p.rho0 + drho;
    const C inv_rho = C(1) / rho;
    const C ux = (jx + C(0.5) * Fx) * inv_rho;
    const C uy = (jy + C(0.5) * Fy) * inv_rho;
    const C uz = (jz + C(0.5) * Fz) * inv_rho;
    const C d3 = drho * C(1.0 / 3.0);
    const C pxx = sxx - d3 - rho * ux * ux, pyy = syy - d3 - rho * uy * uy, pzz = szz - d3 - rho * uz * uz;
    const C pxy = sxy - rho * ux * uy, pxz = sxz - rho * ux * uz, pyz = syz - rho * uy * uz;

    const C qn = sqrt(pxx * pxx + pyy * pyy + pzz * pzz + C(2) * (pxy * pxy + pxz * pxz + pyz * pyz));
    const C tau0 = (C)p.tau;
    C tau_eff = C(0.5) * (tau0 + sqrt(tau0 * tau0 + (C)p.smag_c * qn * inv_rho));
    const bool want = live && tag == LBM_TAG_BGK_MLP;
    if (p.has_mlp && __any(want)) {
        const float feat[7] = {(float)pxx, (float)pyy, (float)pzz, (float)pxy, (float)pxz, (float)pyz, (float)rho};
        const float sp = mlp_wave_eval(p.mlp, feat);
        const C nu0 = (C)p.nu0;
        const C nut = nu0 * (C)sp;
        if (want && isfinite(nut) && nut <= C(10) * nu0) tau_eff = C(3) * (nu0 + nut) + C(0.5);
    }
    const C w = (tag == LBM_TAG_BGK_SMAG || tag == LBM_TAG_BGK_MLP) ? C(1) / tau_eff : (C)p.omega;

    const C uu = ux * ux + uy * uy + uz * uz;
    const C uF = ux * Fx + uy * Fy + uz * Fz;
    const C g = C(1) - C(0.5) * w;
    hs[0] = h[0] - w * (h[0] - C(V<Q, 0>::w) * (drho - C(1.5) * rho * uu)) + g * C(V<Q, 0>::w) * C(-3) * uF;
    sfor<H>([&](auto K) {
        constexpr int k = decltype(K)::value + 1;
        using Vk = V<Q, k>;
        C cu = C(0), cF = C(0);
        if constexpr (Vk::x != 0) cu += C(Vk::x) * ux, cF += C(Vk::x) * Fx;
        if constexpr (Vk::y != 0) cu += C(Vk::y) * uy, cF += C(Vk::y) * Fy;
        if constexpr (Vk::z != 0) cu += C(Vk::z) * uz, cF += C(Vk::z) * Fz;
        const C ev = C(Vk::w) * (drho + rho * (C(4.5) * cu * cu - C(1.5) * uu));
        const C od = C(Vk::w) * C(3) * rho * cu;
        const C Fe = C(Vk::w) * (C(9) * cu * cF - C(3) * uF);
        const C Fo = C(Vk::w) * C(3) * cF;
        const C hp = E[k], hm = O[k];
        const C A = g * Fe - w * (hp - ev);
        const C B = g * Fo - w * (hm - od);
        hs[k] = (hp + hm) + A + B;
        hs[k + H] = (hp - hm) + A - B;
    });
}

// MOM: regularized / recursive-regularized lattices take the moment-only
// update (collide_regularized); the caller decides where that pays.
template <int Q, typename C, int MS, bool MOM = false>
__device__ __forceinline__ void collide_node(const C (&h)[Q], int tag, bool live, const StepParams &p, C (&hs)[Q]) {
    if constexpr (MS == MS_STREAM) {
        // collision switched off: the step only streams (and bounces back)
        sfor<Q>([&](auto I) { hs[decltype(I)::value] = h[decltype(I)::value]; });
        return;
    }
    if constexpr (MOM && (MS == MS_REG || MS == MS_RR)) {
        collide_regularized<Q, C, MS>(h, tag, p, hs);
        return;
    }
    if constexpr (MS == (MS_BGK | MS_SMAG | MS_MLP)) {
        collide_closure<Q, C, MS>(h, tag, live, p, hs);
        return;
    }
    constexpr int H = (Q - 1) / 2;
    C drho = C(0), jx = C(0), jy = C(0), jz = C(0);
    sfor<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        using Vi = V<Q, i>;
        drho += h[i];
        if constexpr (Vi::x == 1) jx += h[i];
        if constexpr (Vi::x == -1) jx -= h[i];
        if constexpr (Vi::y == 1) jy += h[i];
        if constexpr (Vi::y == -1) jy -= h[i];
        if constexpr (Vi::z == 1) jz += h[i];
        if constexpr (Vi::z == -1) jz -= h[i];
    });
    const C Fx = (C)p.force[0], Fy = (C)p.force[1], Fz = (C)p.force[2];
    const C rho = (C)p.rho0 + drho;
    const C inv_rho = C(1) / rho;
    const C ux = (jx + C(0.5) * Fx) * inv_rho;
    const C uy = (jy + C(0.5) * Fy) * inv_rho;
    const C uz = (jz + C(0.5) * Fz) * inv_rho;
    const C uu = ux * ux + uy * uy + uz * uz;
    const C uF = ux * Fx + uy * Fy + uz * Fz;

    // equilibrium, even/odd parts per pair k = 1..H (direction k, opposite k+H)
    C ev[H + 1], od[H + 1], cuk[H + 1];
    ev[0] = C(V<Q, 0>::w) * (drho - C(1.5) * rho * uu);
    od[0] = C(0);
    cuk[0] = C(0);
    sfor<H>([&](auto K) {
        constexpr int k = decltype(K)::value + 1;
        using Vk = V<Q, k>;
        C cu = C(0);
        if constexpr (Vk::x != 0) cu += C(Vk::x) * ux;
        if constexpr (Vk::y != 0) cu += C(Vk::y) * uy;
        if constexpr (Vk::z != 0) cu += C(Vk::z) * uz;
        cuk[k] = cu;
        ev[k] = C(Vk::w) * (drho + rho * (C(4.5) * cu * cu - C(1.5) * uu));
        od[k] = C(Vk::w) * C(3) * rho * cu;
    });

    // relaxation rates from the node's model
    C wp = (C)p.omega, wm = (C)p.omega;
    if constexpr ((MS & MS_TRT) != 0) {
        if (tag == LBM_TAG_TRT) wm = (C)p.omega_minus;
    }
    // Pi_ab = sum c_a c_b (h - heq): only even parts contribute.
    C pxx = C(0), pyy = C(0), pzz = C(0), pxy = C(0), pxz = C(0), pyz = C(0);
    if constexpr ((MS & (MS_SMAG | MS_MLP | MS_REG | MS_RR)) != 0) {
        sfor<H>([&](auto K) {
            constexpr int k = decltype(K)::value + 1;
            using Vk = V<Q, k>;
            const C ne = (h[k] + h[k + H]) - C(2) * ev[k];
            if constexpr (Vk::x != 0) pxx += ne;
            if constexpr (Vk::y != 0) pyy += ne;
            if constexpr (Vk::z != 0) pzz += ne;
            if constexpr (Vk::x * Vk::y != 0) pxy += C(Vk::x * Vk::y) * ne;
            if constexpr (Vk::x * Vk::z != 0) pxz += C(Vk::x * Vk::z) * ne;
            if constexpr (Vk::y * Vk::z != 0) pyz += C(Vk::y * Vk::z) * ne;
        });
    }
    if constexpr ((MS & (MS_SMAG | MS_MLP)) != 0) {
        const C qn = sqrt(pxx * pxx + pyy * pyy + pzz * pzz + C(2) * (pxy * pxy + pxz * pxz + pyz * pyz));
        const C tau0 = (C)p.tau;
        const C tau_s = C(0.5) * (tau0 + sqrt(tau0 * tau0 + (C)p.smag_c * qn * inv_rho));
        C tau_eff = tau_s;
        if constexpr ((MS & MS_MLP) != 0) {
            const bool want = live && tag == LBM_TAG_BGK_MLP;
            if (p.has_mlp && __any(want)) {
                const float feat[7] = {(float)pxx, (float)pyy, (float)pzz, (float)pxy,
                                       (float)pxz, (float)pyz, (float)rho};
                const float sp = mlp_wave_eval(p.mlp, feat);
                const C nu0 = (C)p.nu0;
                const C nut = nu0 * (C)sp;
                if (isfinite(nut) && nut <= C(10) * nu0) {
                    if (tag == LBM_TAG_BGK_MLP) tau_eff = C(3) * (nu0 + nut) + C(0.5);
                }
            }
        }
        if (tag == LBM_TAG_BGK_SMAG || tag == LBM_TAG_BGK_MLP) {
            wp = C(1) / tau_eff;
            wm = wp;
        }
    }

    // Regularized BGK (second-order Hermite projection of the first-order
    // non-equilibrium part, Guo forcing).  The populations read
    // f = feq + f1 - F_i/2, f1 having the momentum flux Pi1 = Pi + (uF + Fu)/2;
    // relaxing feq + w_i Q_i:Pi1 / (2 cs^4) - F_i/2 gives
    //   f*_i = feq_i + (1 - omega) w_i (9/2) (c_i.Pi1.c_i - tr Pi1 / 3) + F_i / 2,
    // which is the omega = 1 update below (A, B) plus the regularized term added
    // to the even part of each pair.
    // Recursive regularized (the paper's RR model, Sec. 3.1-3.2): the same with
    // the deviatoric part of Pi1 only (bulk relaxation 1), i.e. the even term
    // (1 - omega) w_i (9/2) (c_i.Pi1.c_i - |c_i|^2 tr Pi1 / 3), plus the odd
    // third-order Hermite term of T = rho u u u + A3, A3 the recursive
    // non-equilibrium coefficient A3_abc = u_a A2_bc + u_b A2_ac + u_c A2_ab of
    // A2 = (1 - omega) dev Pi1.  Third-order polynomials: the sums and
    // differences of H_xxy and H_yzz, H_xzz and H_xyy, H_yyz and H_xxz
    // (orthogonal on D3Q19 and D3Q27) and, on D3Q27, H_xyz; each projected with
    // its lattice norm (D3Q19: 2/27 for sums, 6/27 for differences; D3Q27: 4/27,
    // and 1/27 for H_xyz).
    C reg = C(0);      // (1 - omega) * 9/2 on regularized nodes, else 0
    C trm = C(1);      // 1 (regularized) or 0 (recursive: its trace is relaxed with 1)
    bool rr = false;   // recursive regularized node
    C rxx = C(0), ryy = C(0), rzz = C(0), rxy = C(0), rxz = C(0), ryz = C(0), rtr = C(0);
    C t1p = C(0), t1m = C(0), t2p = C(0), t2m = C(0), t3p = C(0), t3m = C(0), t7 = C(0);
    if constexpr ((MS & (MS_REG | MS_RR)) != 0) {
        if constexpr ((MS & MS_REG) != 0) {
            if (tag == LBM_TAG_REG) {
                reg = (C(1) - (C)p.omega) * C(4.5);
                wp = C(1);
                wm = C(1);
            }
        }
        if constexpr ((MS & MS_RR) != 0) {
            if (tag == LBM_TAG_RR) {
                reg = (C(1) - (C)p.omega) * C(4.5);
                trm = C(0);
                rr = true;
                wp = C(1);
                wm = C(1);
            }
        }
        rxx = pxx + ux * Fx;
        ryy = pyy + uy * Fy;
        rzz = pzz + uz * Fz;
        rxy = pxy + C(0.5) * (ux * Fy + uy * Fx);
        rxz = pxz + C(0.5) * (ux * Fz + uz * Fx);
        ryz = pyz + C(0.5) * (uy * Fz + uz * Fy);
        rtr = (rxx + ryy + rzz) * C(1.0 / 3.0);
        if constexpr ((MS & MS_RR) != 0) {
            // A2 = (1 - omega) dev Pi1, A3 recursive, T = rho u u u + A3
            const C om1 = C(1) - (C)p.omega;
            const C axx = om1 * (rxx - rtr), ayy = om1 * (ryy - rtr), azz = om1 * (rzz - rtr);
            const C axy = om1 * rxy, axz = om1 * rxz, ayz = om1 * ryz;
            const C txxy = rho * ux * ux * uy + C(2) * ux * axy + uy * axx;
            const C tyzz = rho * uy * uz * uz + uy * azz + C(2) * uz * ayz;
            const C txzz = rho * ux * uz * uz + ux * azz + C(2) * uz * axz;
            const C txyy = rho * ux * uy * uy + ux * ayy + C(2) * uy * axy;
            const C tyyz = rho * uy * uy * uz + C(2) * uy * ayz + uz * ayy;
            const C txxz = rho * ux * ux * uz + C(2) * ux * axz + uz * axx;
            constexpr double np_ = Q == 19 ? 27.0 / 2.0 : 27.0 / 4.0;  // 1 / norm of a sum
            constexpr double nm_ = Q == 19 ? 27.0 / 6.0 : 27.0 / 4.0;  // 1 / norm of a difference
            t1p = (txxy + tyzz) * C(np_);
            t1m = (txxy - tyzz) * C(nm_);
            t2p = (txzz + txyy) * C(np_);
            t2m = (txzz - txyy) * C(nm_);
            t3p = (tyyz + txxz) * C(np_);
            t3m = (tyyz - txxz) * C(nm_);
            if constexpr (Q == 27) t7 = (rho * ux * uy * uz + ux * ayz + uy * axz + uz * axy) * C(27.0);
        }
    }

    const C gp = C(1) - C(0.5) * wp, gm = C(1) - C(0.5) * wm;
    const C F0 = C(V<Q, 0>::w) * C(-3) * uF;
    hs[0] = h[0] - wp * (h[0] - ev[0]) + gp * F0;
    if constexpr ((MS & (MS_REG | MS_RR)) != 0) hs[0] -= reg * C(V<Q, 0>::w) * rtr * trm;
    sfor<H>([&](auto K) {
        constexpr int k = decltype(K)::value + 1;
        using Vk = V<Q, k>;
        C cF = C(0);
        if constexpr (Vk::x != 0) cF += C(Vk::x) * Fx;
        if constexpr (Vk::y != 0) cF += C(Vk::y) * Fy;
        if constexpr (Vk::z != 0) cF += C(Vk::z) * Fz;
        const C Fe = C(Vk::w) * (C(9) * cuk[k] * cF - C(3) * uF);
        const C Fo = C(Vk::w) * C(3) * cF;
        const C hp = C(0.5) * (h[k] + h[k + H]);
        const C hm = C(0.5) * (h[k] - h[k + H]);
        C A = gp * Fe - wp * (hp - ev[k]);
        const C B = gm * Fo - wm * (hm - od[k]);
        C Bx = B;
        if constexpr ((MS & (MS_REG | MS_RR)) != 0) {
            C cpc = C(0);  // c_k . Pi1 . c_k
            if constexpr (Vk::x != 0) cpc += rxx;
            if constexpr (Vk::y != 0) cpc += ryy;
            if constexpr (Vk::z != 0) cpc += rzz;
            if constexpr (Vk::x * Vk::y != 0) cpc += C(2 * Vk::x * Vk::y) * rxy;
            if constexpr (Vk::x * Vk::z != 0) cpc += C(2 * Vk::x * Vk::z) * rxz;
            if constexpr (Vk::y * Vk::z != 0) cpc += C(2 * Vk::y * Vk::z) * ryz;
            // regularized: |c|^2 -> 1 (tr Q = 0 projection); recursive: |c|^2 (deviatoric)
            const C cc = trm + (C(1) - trm) * C(Vk::n2);
            A += reg * C(Vk::w) * (cpc - rtr * cc);
        }
        if constexpr ((MS & MS_RR) != 0) {
            // odd third-order Hermite term (both equilibrium and non-equilibrium)
            constexpr int cx = Vk::x, cy = Vk::y, cz = Vk::z;
            constexpr double p1p = cy * (cx * cx + cz * cz - 2.0 / 3.0), p1m = cy * (cx * cx - cz * cz);
            constexpr double p2p = cx * (cy * cy + cz * cz - 2.0 / 3.0), p2m = cx * (cz * cz - cy * cy);
            constexpr double p3p = cz * (cx * cx + cy * cy - 2.0 / 3.0), p3m = cz * (cy * cy - cx * cx);
            constexpr double p7 = cx * cy * cz;
            C e3 = C(0);
            if constexpr (p1p != 0.0) e3 += C(p1p) * t1p;
            if constexpr (p1m != 0.0) e3 += C(p1m) * t1m;
            if constexpr (p2p != 0.0) e3 += C(p2p) * t2p;
            if constexpr (p2m != 0.0) e3 += C(p2m) * t2m;
            if constexpr (p3p != 0.0) e3 += C(p3p) * t3p;
            if constexpr (p3m != 0.0) e3 += C(p3m) * t3m;
            if constexpr (Q == 27 && p7 != 0.0) e3 += C(p7) * t7;
            if (rr) Bx += C(Vk::w) * e3;
        }
        hs[k] = h[k] + A + Bx;
        hs[k + H] = h[k + H] + A - Bx;
    });

    if constexpr ((MS & MS_OPEN) != 0) {
        if (tag >= LBM_TAG_VEL_IN && tag <= LBM_TAG_VEL_OUT) open_boundary<Q, C>(h, tag, p, hs);
    }
}

// The fused collide-and-stream step: one thread per node, 256-thread blocks
// covering a tile of (1 << tx_log2) x (256 >> tx_log2) nodes of one z-plane.
// Wall handling selects addresses rather than branching around loads, so the
// Q loads of a thread are all in flight together.
template <int Q, int P, int MS, bool TAGGED, int MODE, int PARITY, int ADDR>
__global__ __launch_bounds__(256) void k_collide_stream(StepParams p) {
    using S = typename Prec<P>::S;
    using C = typename Prec<P>::C;
    // ADDR 0: row layout, node-form addresses; 1: row layout, row-form
    // addresses; 2: brick layout (tagged kernels), node-form addresses
    constexpr bool ROWS = ADDR == 1;
    constexpr bool BRICK = ADDR == 2;

    // XCD-aware tile order: hardware deals workgroups round-robin over the 8
    // XCDs, so workgroup w runs on XCD w % 8; give each XCD a contiguous run
    // of tiles (whole z-slabs) so neighbouring rows share that XCD's L2.
    const int wg = blockIdx.x;
    const int L = (wg & 7) * p.tiles_per_xcd + (wg >> 3);
    if (L >= p.n_tiles) return;  // uniform for the block

    const int nx = p.nx, ny = p.ny, nz = p.nz;
    int x, y, z;
    bool brick_none = false;  // brick layout: a padding wave past the last listed brick
    int xo[3], yo[3], zo[3];  // storage-index terms of the neighbours, index 1 + c for c in {-1, 0, 1}
    if constexpr (!BRICK) {
        // row layout: a tile of (1 << tx_log2) x (256 >> tx_log2) nodes of one plane
        const int txl = p.tx_log2;
        const int TX = 1 << txl, TY = 256 >> txl;
        const int tix = L % p.tiles_x;
        const int rem = L / p.tiles_x;
        const int tiy = rem % p.tiles_y;
        z = rem / p.tiles_y;
        x = (tix << txl) + (threadIdx.x & (TX - 1));
        y = tiy * TY + (threadIdx.x >> txl);
        // neighbour offsets with periodic wrap
        const bool in = (x < nx) && (y < ny);
        const int xc = in ? x : 0, yc = in ? y : 0;
        xo[0] = xc == 0 ? nx - 1 : xc - 1, xo[1] = xc, xo[2] = xc + 1 == nx ? 0 : xc + 1;
        yo[0] = (yc == 0 ? ny - 1 : yc - 1) * nx, yo[1] = yc * nx, yo[2] = (yc + 1 == ny ? 0 : yc + 1) * nx;
        const int nxy = nx * ny;
        zo[0] = (z == 0 ? nz - 1 : z - 1) * nxy, zo[1] = z * nxy, zo[2] = (z + 1 == nz ? 0 : z + 1) * nxy;
    } else {
        // brick layout: wave w of tile L updates the brick listed at [L][w] (the
        // bricks that hold fluid, in storage order, so solid rock launches no
        // wave), lane l the node (l % 4, l / 4 % 4, l / 16) of that brick; brick
        // b is brick b % 64 of 16^3 block b / 64 (every axis a multiple of 16)
        typedef const __attribute__((address_space(4))) int const_int;
        const int l = threadIdx.x & 63;
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const int b = ((const_int *)p.tile_tag)[L * 4 + wave];
        brick_none = b < 0;
        const int bb = brick_none ? 0 : b;
        const int blk = bb >> 6, bib = bb & 63;
        const Layout &ly = p.lay;
        const int bz = blk / ly.nbxy, brem = blk - bz * ly.nbxy;
        const int by = brem / ly.nbx, bx = brem - by * ly.nbx;
        x = bx * 16 + (bib & 3) * 4 + (l & 3);
        y = by * 16 + ((bib >> 2) & 3) * 4 + ((l >> 2) & 3);
        z = bz * 16 + (bib >> 4) * 4 + (l >> 4);
        xo[0] = ly.x(x == 0 ? nx - 1 : x - 1), xo[1] = ly.x(x), xo[2] = ly.x(x + 1 == nx ? 0 : x + 1);
        yo[0] = ly.y(y == 0 ? ny - 1 : y - 1), yo[1] = ly.y(y), yo[2] = ly.y(y + 1 == ny ? 0 : y + 1);
        zo[0] = ly.z(z == 0 ? nz - 1 : z - 1), zo[1] = ly.z(z), zo[2] = ly.z(z + 1 == nz ? 0 : z + 1);
    }
    const bool active = (x < nx) && (y < ny);
    const int n = zo[1] + yo[1] + xo[1];  // storage index of the node

    // Node class.  Waves whose 64 nodes and their one-node halo are a single
    // fluid model (the interior of a walled domain) need nothing; waves with no
    // fluid or filler node (solid rock) skip the update; the other waves read
    // each node's precomputed neighbour mask (wave-uniform branches).
    S *__restrict__ f = static_cast<S *>(p.pops);
    const long long pb = pop_base<Q>(n);
    int tag = p.uniform_tag;
    uint32_t wall = 0;   // bit i: node x + c_i is not fluid
    bool moving = false; // some neighbour is a moving wall
    bool plain = !TAGGED;
    bool skip = false;
    if constexpr (TAGGED) {
        // wave-uniform entry read through the constant address space (scalar load)
        typedef const __attribute__((address_space(4))) int const_int;
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const int tile_tag = BRICK ? (brick_none ? -1 : 0) : ((const_int *)p.tile_tag)[L * 4 + wave];
        if (tile_tag > 0) {
            tag = tile_tag;
            plain = true;
        } else if (tile_tag < 0) {
            tag = 0;
            skip = true;
        } else {
            const uint32_t m = active ? p.mask[n] : 0u;
            wall = m & kMaskWalls;
            moving = (m >> kMaskMovingBit) & 1u;
            tag = (int)(m >> kMaskTagShift);
        }
    }
    const bool live = active && (!TAGGED || tag != 0);
    // Filler stores.  A non-fluid node that shares a 64-byte storage sector with
    // fluid nodes stores into slots no fluid node reads or writes, so that the
    // sectors the step writes are written whole instead of partially (partial
    // sectors cost the memory a read-modify-write): in the even step its own
    // slots; in the odd step slot i of node x + (0, c_iy, c_iz) when that node
    // is not fluid (the row the wave's other lanes write for direction i).
    // Its loaded values are zero and its stored values are never read.
    const bool filler = TAGGED && active && tag == 0 && (wall & 1u);

    double red[NRED];
    if constexpr (MODE != MODE_STEP) {
#pragma unroll
        for (int k = 0; k < NRED; ++k) red[k] = 0.0;
    }

    // The node update with either of two address forms.  Row form (ROWS
    // variants; which waves use it is chosen below): whole rows tile the
    // 4096-node blocks and the tile is at least a wave wide (the host checks
    // both), so the wave's 64 nodes lie in one row and each population row it
    // reads or writes starts at a wave-uniform address: a scalar base plus the
    // lane's x offset, no per-lane 64-bit address arithmetic (wall waves
    // select per lane between two such addresses).  Node form: every address
    // computed per node, with wall selection.
    auto update = [&](auto rows_c, auto walls_c) {
        constexpr bool RF = decltype(rows_c)::value;     // row form
        constexpr bool WALLS = decltype(walls_c)::value; // wall, filler and moving-wall code
        // row form: population 0 at x = 0 of row (y + dy, z + dz), index [1 + dz][1 + dy],
        // and the lane's byte offsets of x - 1, x, x + 1 (periodic)
        const S *rp[3][3] = {};
        unsigned xb[3] = {0u, 0u, 0u};
        if constexpr (RF) {
            const int ys = __builtin_amdgcn_readfirstlane(y);
            const int yv[3] = {ys == 0 ? ny - 1 : ys - 1, ys, ys + 1 == ny ? 0 : ys + 1};
            const int zv[3] = {z == 0 ? nz - 1 : z - 1, z, z + 1 == nz ? 0 : z + 1};
            const int rl = p.row_log2;
            sfor<3>([&](auto DZ) {
                sfor<3>([&](auto DY) {
                    constexpr int dz = decltype(DZ)::value, dy = decltype(DY)::value;
                    if (PARITY == 1 || (dz == 1 && dy == 1)) {
                        const int r = zv[dz] * ny + yv[dy];
                        rp[dz][dy] = f + (long long)(r >> rl) * (long long)(Q << kBlockLog2) +
                                     (long long)((r & ((1 << rl) - 1)) * nx);
                    }
                });
            });
#pragma unroll
            for (int k = 0; k < 3; ++k) xb[k] = (unsigned)xo[k] * (unsigned)sizeof(S);
        }
        // Slot base in scalar registers (wave-uniform: the row bases derive from
        // the wave's row; the empty asm keeps the compiler from re-associating
        // the slot offset into per-lane 64-bit adds), plus the lane's 32-bit
        // offset: one global access with a scalar base.
        typedef __attribute__((address_space(1))) S gS;
        typedef __attribute__((address_space(1))) char gchar;
        auto at = [&](const S *row, int slot, unsigned xoff) -> gS * {
            gS *b = (gS *)(row + slot_off(slot));
            asm("" : "+s"(b));
            return (gS *)((gchar *)b + xoff);
        };

        // ---- pull the node's populations.  The registers are zeroed first and the
        // loads sit in a branch with no else: a divergent else that overwrote
        // registers with loads in flight would force a wait on those loads.
        C h[Q];
        sfor<Q>([&](auto I) { h[decltype(I)::value] = C(0); });
        if (live) {
            sfor<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                using Vi = V<Q, i>;
                if constexpr (RF) {
                    if constexpr (PARITY == 0 || i == 0) {
                        h[i] = (C)*at(rp[1][1], i, xb[1]);
                    } else {
                        gS *a = at(rp[1 - Vi::z][1 - Vi::y], Vi::opp, xb[1 - Vi::x]);
                        if constexpr (WALLS) {
                            // a wall at x - c_i: the node's own slot i instead
                            gS *own = at(rp[1][1], i, xb[1]);
                            a = ((wall >> Vi::opp) & 1u) ? own : a;
                        }
                        h[i] = (C)*a;
                    }
                } else {
                    long long off;
                    if constexpr (PARITY == 0 || i == 0) {
                        off = pb + slot_off(i);
                    } else {
                        // direction i arrives from x - c_i (slot opp), or from the node's
                        // own slot i when x - c_i is a wall
                        const long long o_nb =
                            pop_base<Q>(zo[1 - Vi::z] + yo[1 - Vi::y] + xo[1 - Vi::x]) + slot_off(Vi::opp);
                        if constexpr (TAGGED) {
                            off = ((wall >> Vi::opp) & 1u) ? pb + slot_off(i) : o_nb;
                        } else {
                            off = o_nb;
                        }
                    }
                    h[i] = (C)f[off];
                }
            });
        }

        if constexpr (MODE != MODE_STEP) node_reduce<Q, C>(h, live, p, red);

        if constexpr (MODE != MODE_REDUCE) {
            C hs[Q];
            // moment-only regularized update in FP16 storage and FP64 (fewer
            // registers: FP16 +10-14%, FP64 RR +4%); FP32 measured 0.5-2%
            // slower with it and keeps the general update
            collide_node<Q, C, MS, P != 1>(h, tag, live, p, hs);

            // moving-wall term where x + c_i is a moving wall (nodes next to one only)
            if constexpr (TAGGED && WALLS) {
                if (moving) {
                    sfor<Q>([&](auto I) {
                        constexpr int i = decltype(I)::value;
                        using Vi = V<Q, i>;
                        if constexpr (i > 0) {
                            if ((wall >> i) & 1u) {
                                const int dst = zo[1 + Vi::z] + yo[1 + Vi::y] + xo[1 + Vi::x];
                                const int t = p.tags[dst];
                                if (t >= LBM_TAG_WALL0) {
                                    const double *uw = p.wall_u + 3 * (t - LBM_TAG_WALL0);
                                    C cu = C(0);
                                    if constexpr (Vi::x != 0) cu += C(Vi::x) * (C)uw[0];
                                    if constexpr (Vi::y != 0) cu += C(Vi::y) * (C)uw[1];
                                    if constexpr (Vi::z != 0) cu += C(Vi::z) * (C)uw[2];
                                    hs[i] -= C(6.0 * Vi::w) * (C)p.rho0 * cu;
                                }
                            }
                        }
                    });
                }
            }

            // ---- push
            if constexpr (RF) {
                if (live || (WALLS && filler)) {
                    sfor<Q>([&](auto I) {
                        constexpr int i = decltype(I)::value;
                        using Vi = V<Q, i>;
                        if constexpr (i == 0) {
                            *at(rp[1][1], 0, xb[1]) = (S)hs[0];
                        } else if constexpr (PARITY == 0) {
                            *at(rp[1][1], Vi::opp, xb[1]) = (S)hs[i];
                        } else if constexpr (!WALLS) {
                            *at(rp[1 + Vi::z][1 + Vi::y], i, xb[1 + Vi::x]) = (S)hs[i];
                        } else {
                            // a wall at x + c_i: back to the node's own slot opp(i), or
                            // (filler) slot i of x + (0, c_iy, c_iz)
                            gS *a = at(rp[1 + Vi::z][1 + Vi::y], i, xb[1 + Vi::x]);
                            const bool wi = (wall >> i) & 1u;
                            gS *alt = live ? at(rp[1][1], Vi::opp, xb[1]) : at(rp[1 + Vi::z][1 + Vi::y], i, xb[1]);
                            a = wi ? alt : a;
                            if (live || wi) *a = (S)hs[i];
                        }
                    });
                }
            } else if (live || filler) {
                sfor<Q>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    using Vi = V<Q, i>;
                    long long off;
                    bool ok = true;
                    if constexpr (i == 0) {
                        off = pb;
                    } else if constexpr (PARITY == 0) {
                        // even step: h*_i goes to slot opp(i) of the node itself
                        off = pb + slot_off(Vi::opp);
                    } else {
                        // odd step: h*_i goes to slot i of x + c_i, or back to slot
                        // opp(i) of the node itself when x + c_i is a wall
                        off = pop_base<Q>(zo[1 + Vi::z] + yo[1 + Vi::y] + xo[1 + Vi::x]) + slot_off(i);
                        if constexpr (TAGGED) {
                            const bool wi = (wall >> i) & 1u;
                            if (wi) off = live ? pb + slot_off(Vi::opp)
                                               : pop_base<Q>(zo[1 + Vi::z] + yo[1 + Vi::y] + xo[1]) + slot_off(i);
                            ok = live || wi;
                        }
                    }
                    if (ok) f[off] = (S)hs[i];
                });
            }
        }
    };
    using yes = std::true_type;
    using no = std::false_type;
    if constexpr (ROWS && !TAGGED) {
        update(yes{}, no{});
    } else if (skip) {
        // no fluid or filler node: nothing to load, update or store
    } else if constexpr (ROWS && P == 2) {
        if (plain) update(yes{}, no{});
        else update(yes{}, yes{});
    } else if constexpr (ROWS) {
        if (plain) update(no{}, yes{});
        else update(yes{}, yes{});
    } else {
        update(no{}, std::integral_constant<bool, TAGGED>{});
    }

    // ---- per-tile reduction partials (fixed order: shuffle tree, then waves 0..3)
    if constexpr (MODE != MODE_STEP) {
        __shared__ double s_red[4][NRED];
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
        for (int k = 0; k < NRED; ++k) {
            double v = red[k];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
            if (lane == 0) s_red[wave][k] = v;
        }
        __syncthreads();
        if (threadIdx.x < NRED) {
            const int k = threadIdx.x;
            p.partials[(long long)k * p.partial_stride + L] = (s_red[0][k] + s_red[1][k]) + (s_red[2][k] + s_red[3][k]);
        }
    }
}

// ---- FP16 storage, two nodes per lane (even step)
//
// Lattices of one fluid model without walls (untagged), stored in FP16, whose
// rows of 128..4096 nodes tile the 4096-node blocks.  Wave w of tile L updates
// the 128-node row segment 4 L + w, lane l its nodes x0 = 2 l and x0 + 1 from
// the segment start, reading and writing each population row with aligned
// 4-byte accesses (a wave moves 256 contiguous bytes per row instead of 128).
// The even step only: every access stays at the nodes themselves (an odd step
// in this form, its x-shifted rows combined across lanes with DPP shifts, ran
// slower than the one-node odd step at two waves per SIMD).  The node update is
// the one-node code run twice; where the compiler shares a product between the
// two nodes it may fuse one multiply-add fewer, so a rare population differs
// from the one-node kernels' by one FP16 rounding.
__device__ __forceinline__ float half_lo(uint32_t v) {
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(v & 0xffffu));
}
__device__ __forceinline__ float half_hi(uint32_t v) { return (float)__builtin_bit_cast(_Float16, (unsigned short)(v >> 16)); }
__device__ __forceinline__ uint32_t half_bits(float v) { return (uint32_t)__builtin_bit_cast(unsigned short, (_Float16)v); }

template <int Q, int MS>
__global__ __launch_bounds__(256) void k_collide_pair_even(StepParams p) {
    using C = float;
    // tiles of four segments, dealt to the XCDs in contiguous runs (as k_collide_stream)
    const int n_tiles = (p.n_segs + 3) >> 2;
    const int per_xcd = (n_tiles + 7) >> 3;
    const int wg = blockIdx.x;
    const int L = (wg & 7) * per_xcd + (wg >> 3);
    if (L >= n_tiles) return;  // uniform for the block
    const int sg = L * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (sg >= p.n_segs) return;  // uniform for the wave (the last tile may be short)
    const int lane = threadIdx.x & 63;
    const int nx = p.nx;
    const long long s0 = (long long)sg * 128;  // natural index of the segment's first node
    const int nxl = __builtin_ctz((unsigned)nx);
    const int xs = (int)(s0 & (nx - 1));
    const int r = (int)(s0 >> nxl);            // row z ny + y
    const int rl = p.row_log2;
    // population 0 at x = 0 of the row, and the lane's byte offset in it
    _Float16 *__restrict__ f = static_cast<_Float16 *>(p.pops);
    const _Float16 *row =
        f + (long long)(r >> rl) * (long long)(Q << kBlockLog2) + (long long)((r & ((1 << rl) - 1)) * nx);
    const unsigned xb = (unsigned)(xs + 2 * lane) * 2u;
    typedef __attribute__((address_space(1))) uint32_t gU32;
    typedef __attribute__((address_space(1))) char gchar;
    auto at = [&](int slot) -> gU32 * {
        gchar *b = (gchar *)(row + slot_off(slot));
        asm("" : "+s"(b));  // scalar base, lane offset added per access
        return (gU32 *)(b + xb);
    };

    // u[i]: h_i of both nodes (low half: x0, high half: x0 + 1)
    uint32_t u[Q], o[Q];
    sfor<Q>([&](auto I) { u[decltype(I)::value] = *at(decltype(I)::value); });
    const int tag = p.uniform_tag;
    sfor<2>([&](auto K) {
        constexpr int k = decltype(K)::value;
        C h[Q], hs[Q];
        sfor<Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            h[i] = k == 0 ? half_lo(u[i]) : half_hi(u[i]);
        });
        collide_node<Q, C, MS, true>(h, tag, true, p, hs);
        sfor<Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            if constexpr (k == 0) o[i] = half_bits(hs[i]);
            else o[i] |= half_bits(hs[i]) << 16;
        });
    });
    // h*_i to slot opp(i) of the nodes themselves
    sfor<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        *at(V<Q, i>::opp) = o[i];
    });
}

// Neighbour mask of every node (see kMask*): wall bits, moving-wall flag and
// the node's own fluid tag (0 for non-fluid nodes); tags and masks in storage
// order (lay).
template <int Q>
__global__ __launch_bounds__(256) void k_build_mask(const uint8_t *tags, int nx, int ny, int nz, Layout lay,
                                                    int sector_log2, int odd_fill, uint32_t *mask) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long N = (long long)nx * ny * nz;
    if (t >= N) return;
    const int x = (int)(t % nx), y = (int)((t / nx) % ny), z = (int)(t / ((long long)nx * ny));
    auto fluid_at = [&](int gx, int gy, int gz) { return is_fluid_tag(tags[lay.at(gx, gy, gz)]); };
    const long long s = lay.at(x, y, z);
    const int own = tags[s];
    uint32_t m = 0;
    if (is_fluid_tag(own)) {
        m = (uint32_t)own << kMaskTagShift;
        sfor<Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            if constexpr (i > 0) {
                using Vi = V<Q, i>;
                const int gx = wrap_idx(x + Vi::x, nx), gy = wrap_idx(y + Vi::y, ny), gz = wrap_idx(z + Vi::z, nz);
                const int tn = tags[lay.at(gx, gy, gz)];
                if (!is_fluid_tag(tn)) m |= 1u << i;
                if (tn >= LBM_TAG_WALL0) m |= 1u << kMaskMovingBit;
            }
        });
    } else {
        // filler: a non-fluid node in a storage sector that also holds fluid nodes
        const long long g = 1ll << sector_log2;
        const long long a = s & ~(g - 1), b = a + g < N ? a + g : N;
        bool any = false;
        for (long long k = a; k < b; ++k) any |= is_fluid_tag(tags[k]);
        if (any) {
            m = 1u;
            if (odd_fill) {
                sfor<Q>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    if constexpr (i > 0) {
                        using Vi = V<Q, i>;
                        if (!fluid_at(x, wrap_idx(y + Vi::y, ny), wrap_idx(z + Vi::z, nz))) m |= 1u << i;
                    }
                });
            }
        }
    }
    mask[s] = m;
}

// ------------------------------------------------------------- helpers

// Storage index of the node with natural index n = (z ny + y) nx + x.
__device__ __forceinline__ int storage_index(const AuxParams &a, long long n) {
    if (!a.lay.brick) return (int)n;
    const int x = (int)(n % a.nx), y = (int)((n / a.nx) % a.ny), z = (int)(n / ((long long)a.nx * a.ny));
    return a.lay.at(x, y, z);
}

// Equilibrium initialisation (FP64 arithmetic, rounded once to storage).
template <int Q, int P>
__global__ __launch_bounds__(256) void k_init(AuxParams a) {
    using S = typename Prec<P>::S;
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= a.count) return;
    const int n = storage_index(a, a.cell0 + t);
    if (!is_fluid_tag(a.tags[n])) return;
    const double rho = a.in_rho ? a.in_rho[t] : a.rho0;
    const double ux = a.in_u ? a.in_u[t] : 0.0;
    const double uy = a.in_u ? a.in_u[a.count + t] : 0.0;
    const double uz = a.in_u ? a.in_u[2 * a.count + t] : 0.0;
    const double drho = rho - a.rho0;
    const double uu = ux * ux + uy * uy + uz * uz;
    S *f = static_cast<S *>(a.pops);
    sfor<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        using Vi = V<Q, i>;
        const double cu = Vi::x * ux + Vi::y * uy + Vi::z * uz;
        const double heq = Vi::w * (drho + rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
        f[pop_base<Q>(n) + slot_off(i)] = (S)heq;
    });
}

// Natural state of the node with natural index n: h_i(n) for every i (slot
// map of the layout parity).
template <int Q, int P>
__device__ __forceinline__ void load_natural(const AuxParams &a, long long n, double (&fo)[Q]) {
    using S = typename Prec<P>::S;
    const S *f = static_cast<const S *>(a.pops);
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((long long)nx * ny));
    const int sn = a.lay.at(x, y, z);
    sfor<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        using Vi = V<Q, i>;
        long long off = pop_base<Q>(sn) + slot_off(i);
        if (a.parity != 0 && i != 0) {
            const int sx = wrap_idx(x - Vi::x, nx), sy = wrap_idx(y - Vi::y, ny), sz = wrap_idx(z - Vi::z, nz);
            const int src = a.lay.at(sx, sy, sz);
            if (is_fluid_tag(a.tags[src])) off = pop_base<Q>(src) + slot_off(Vi::opp);
        }
        fo[i] = a.shifted ? (double)f[off] : (double)f[off] + Vi::w * a.rho0;
    });
}

template <int Q, int P>
__global__ __launch_bounds__(256) void k_gather(AuxParams a, int gmode) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= a.count) return;
    const long long n = gmode == G_CELLS ? a.cells[t] : a.cell0 + t;
    const bool fl = is_fluid_tag(a.tags[storage_index(a, n)]);
    if (gmode == G_FIELDS) a.shifted = 0;
    double fo[Q];
    if (fl) {
        load_natural<Q, P>(a, n, fo);
    } else {
        sfor<Q>([&](auto I) { fo[decltype(I)::value] = 0.0; });
    }
    if (gmode == G_POPS) {
        sfor<Q>([&](auto I) { a.out[(long long)decltype(I)::value * a.count + t] = fo[decltype(I)::value]; });
    } else if (gmode == G_CELLS) {
        sfor<Q>([&](auto I) { a.out[t * Q + decltype(I)::value] = fo[decltype(I)::value]; });
    } else {
        double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
        sfor<Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            using Vi = V<Q, i>;
            rho += fo[i];
            jx += Vi::x * fo[i];
            jy += Vi::y * fo[i];
            jz += Vi::z * fo[i];
        });
        const double inv = fl ? 1.0 / rho : 0.0;
        a.out[t] = rho;
        a.out[a.count + t] = fl ? (jx + 0.5 * a.force[0]) * inv : 0.0;
        a.out[2 * a.count + t] = fl ? (jy + 0.5 * a.force[1]) * inv : 0.0;
        a.out[3 * a.count + t] = fl ? (jz + 0.5 * a.force[2]) * inv : 0.0;
    }
}

// Write natural-layout populations (unshifted FP64 in, shifted storage out).
template <int Q, int P>
__global__ __launch_bounds__(256) void k_scatter(AuxParams a) {
    using S = typename Prec<P>::S;
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= a.count) return;
    const int n = storage_index(a, a.cell0 + t);
    if (!is_fluid_tag(a.tags[n])) return;
    S *f = static_cast<S *>(a.pops);
    sfor<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        using Vi = V<Q, i>;
        const double v = a.in_f[(long long)i * a.count + t];
        f[pop_base<Q>(n) + slot_off(i)] = (S)(a.shifted ? v : v - Vi::w * a.rho0);
    });
}

// Slab-face copy: one thread per node of the plane; each copies the slots of
// the directions crossing the face (c_z = +1 on face 0, c_z = -1 on face 1),
// the j-th of them to buf[j][y][x].  Coalesced along x on both sides.
template <int Q, int P>
__global__ __launch_bounds__(256) void k_face(AuxParams a, int face, int unpack, void *buf) {
    using S = typename Prec<P>::S;
    const long long nxy = (long long)a.nx * a.ny;
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= nxy) return;
    const int plane = face == 0 ? 0 : a.nz - 1;
    const int n = storage_index(a, (long long)plane * nxy + t);
    S *f = static_cast<S *>(a.pops);
    S *b = static_cast<S *>(buf);
    const long long base = pop_base<Q>(n);
    const int cz = face == 0 ? 1 : -1;
    int j = 0;
    sfor<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if constexpr (V<Q, i>::z != 0) {
            if (V<Q, i>::z == cz) {
                S *slot = f + base + slot_off(i);
                S *e = b + (long long)j * nxy + t;
                if (unpack) *slot = *e;
                else *e = *slot;
                ++j;
            }
        }
    });
}

// ------------------------------------------------------------- launchers

// Dynamic LDS that the even-step kernel of FP32/FP64 row-form (walled,
// mostly fluid) lattices does not use: it caps a CU's 160 KB of LDS at three
// workgroups, i.e. three waves per SIMD.  Measured on the 256^3 cavity: FP32
// +1.0% (two waves per SIMD: -2%), FP64 +0.2%, regularized +0.4-0.6%; FP16
// and the odd step lose with any cap.
constexpr unsigned kEvenLdsCap = 41u << 10;

template <int Q, int P, int MS, bool TG, int MODE, int ADDR>
static hipError_t launch_step_rows(const StepParams &p, int parity, hipStream_t s) {
    const dim3 grid(8 * p.tiles_per_xcd), block(256);
    constexpr unsigned lds_even = (ADDR == 1 && TG && P != 2) ? kEvenLdsCap : 0u;
    if (parity == 0)
        k_collide_stream<Q, P, MS, TG, MODE, 0, ADDR><<<grid, block, lds_even, s>>>(p);
    else
        k_collide_stream<Q, P, MS, TG, MODE, 1, ADDR><<<grid, block, 0, s>>>(p);
    return hipGetLastError();
}

// Row-form variants (see k_collide_stream) where the lattice allows them: in
// FP16 storage for every wave (there the node form's per-lane address
// arithmetic limits the step, the odd step most), in FP32/FP64 for the wall
// waves of tagged lattices only (their selects get cheaper; for plain waves
// and untagged lattices, bound by memory alone, the row form measured 0.5-3%
// slower than the node form).
template <int Q, int P, int MS, bool TG, int MODE>
static hipError_t launch_step_par(const StepParams &p, int parity, hipStream_t s) {
    if constexpr (TG) {
        if (p.lay.brick) return launch_step_rows<Q, P, MS, TG, MODE, 2>(p, parity, s);
    }
    if constexpr (P == 2 && !TG && (MS & MS_MLP) == 0 && MODE == MODE_STEP) {
        // the even step of FP16 lattices of one model: two nodes per lane
        if (p.pair && parity == 0) {
            const int n_tiles = (p.n_segs + 3) / 4;
            k_collide_pair_even<Q, MS><<<dim3(8 * ((n_tiles + 7) / 8)), dim3(256), 0, s>>>(p);
            return hipGetLastError();
        }
    }
    constexpr bool kRows = P == 2 || TG;
    if constexpr (kRows) {
        if (p.row_log2 >= 0) return launch_step_rows<Q, P, MS, TG, MODE, 1>(p, parity, s);
    }
    return launch_step_rows<Q, P, MS, TG, MODE, 0>(p, parity, s);
}

template <int Q, int P, int MS, bool TG>
static hipError_t launch_step_mode(const StepParams &p, int mode, int parity, hipStream_t s) {
    switch (mode) {
        case MODE_STEP: return launch_step_par<Q, P, MS, TG, MODE_STEP>(p, parity, s);
        case MODE_STEP_REDUCE: return launch_step_par<Q, P, MS, TG, MODE_STEP_REDUCE>(p, parity, s);
        default: return launch_step_par<Q, P, MS_BGK, TG, MODE_REDUCE>(p, parity, s);
    }
}

template <int Q, int P, bool TG>
static hipError_t launch_step_ms(const StepParams &p, int ms, int mode, int parity, hipStream_t s) {
    switch (ms) {
        case MS_BGK: return launch_step_mode<Q, P, MS_BGK, TG>(p, mode, parity, s);
        case MS_TRT: return launch_step_mode<Q, P, MS_TRT, TG>(p, mode, parity, s);
        case MS_BGK | MS_SMAG: return launch_step_mode<Q, P, MS_BGK | MS_SMAG, TG>(p, mode, parity, s);
        case MS_BGK | MS_SMAG | MS_MLP: return launch_step_mode<Q, P, MS_BGK | MS_SMAG | MS_MLP, TG>(p, mode, parity, s);
        case MS_REG: return launch_step_mode<Q, P, MS_REG, TG>(p, mode, parity, s);
        case MS_TRT | MS_OPEN: return launch_step_mode<Q, P, MS_TRT | MS_OPEN, TG>(p, mode, parity, s);
        case MS_RR: return launch_step_mode<Q, P, MS_RR, TG>(p, mode, parity, s);
        case kAllModels: return launch_step_mode<Q, P, kAllModels, TG>(p, mode, parity, s);
        case MS_STREAM: return launch_step_mode<Q, P, MS_STREAM, TG>(p, mode, parity, s);
        default: return hipErrorInvalidValue;
    }
}

template <int Q, int P>
hipError_t launch_step(const StepParams &p, int ms, bool tagged, int mode, int parity, hipStream_t s) {
    return tagged ? launch_step_ms<Q, P, true>(p, ms, mode, parity, s)
                  : launch_step_ms<Q, P, false>(p, ms, mode, parity, s);
}

template <int Q>
hipError_t launch_build_mask(const uint8_t *tags, int nx, int ny, int nz, Layout lay, int sector_log2,
                             int odd_fill, uint32_t *mask, hipStream_t s) {
    const long long N = (long long)nx * ny * nz;
    k_build_mask<Q><<<(unsigned)((N + 255) / 256), 256, 0, s>>>(tags, nx, ny, nz, lay, sector_log2, odd_fill, mask);
    return hipGetLastError();
}

template <int Q, int P>
hipError_t launch_init(const AuxParams &a, hipStream_t s) {
    const unsigned blocks = (unsigned)((a.count + 255) / 256);
    k_init<Q, P><<<blocks, 256, 0, s>>>(a);
    return hipGetLastError();
}

template <int Q, int P>
hipError_t launch_gather(const AuxParams &a, int gmode, hipStream_t s) {
    const unsigned blocks = (unsigned)((a.count + 255) / 256);
    k_gather<Q, P><<<blocks, 256, 0, s>>>(a, gmode);
    return hipGetLastError();
}

template <int Q, int P>
hipError_t launch_scatter(const AuxParams &a, hipStream_t s) {
    const unsigned blocks = (unsigned)((a.count + 255) / 256);
    k_scatter<Q, P><<<blocks, 256, 0, s>>>(a);
    return hipGetLastError();
}

template <int Q, int P>
hipError_t launch_face(const AuxParams &a, int face, int unpack, void *buf, hipStream_t s) {
    const long long nxy = (long long)a.nx * a.ny;
    k_face<Q, P><<<(unsigned)((nxy + 255) / 256), 256, 0, s>>>(a, face, unpack, buf);
    return hipGetLastError();
}

#define LBMD_INSTANTIATE(Q, P)                                                                           \
    template hipError_t launch_step<Q, P>(const StepParams &, int, bool, int, int, hipStream_t);          \
    template hipError_t launch_init<Q, P>(const AuxParams &, hipStream_t);                                \
    template hipError_t launch_gather<Q, P>(const AuxParams &, int, hipStream_t);                         \
    template hipError_t launch_scatter<Q, P>(const AuxParams &, hipStream_t);                             \
    template hipError_t launch_face<Q, P>(const AuxParams &, int, int, void *, hipStream_t);

}  // namespace lbmd
