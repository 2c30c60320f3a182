// Device-side cut arithmetic of the Segment Linking chain (gfx950).
//
// The paper (arXiv:2209.13711) prints no formula; these are this project's
// readings of its rules: a stub window equivalent to p_T >= 0.8 GeV (Sec. 2);
// links along +-q helices of threshold p_T from the centre and a relative
// angle between linked objects (Sec. 2.1); triplets and quintuplets from
// objects sharing a stub (Sec. 2.1).
//
// Every expression is parenthesised in the operation order that defines the
// FP32 result.  The library is built with -ffp-contract=off (no FMA
// contraction) and HIP's default correctly rounded division and square root,
// so each operation rounds exactly once and the result is reproducible
// bit for bit on any IEEE-754 binary32 implementation.  min/max are the
// ternaries below and every cut is "lhs <= rhs", so NaN fails.
#pragma once

#include "lst_internal.hpp"

namespace lst {

__device__ __forceinline__ float mn(float a, float b) { return a < b ? a : b; }
__device__ __forceinline__ float mx(float a, float b) { return a > b ? a : b; }

// asin(x)/x at x^2 = x2 (x2 clamped to 0.81): Maclaurin series to x^10 with
// the remaining tail bounded by c6 x^12 / (1 - x^2).
__device__ __forceinline__ float asinx(float x2)
{
    const float A1 = 1.0f / 6.0f, A2 = 3.0f / 40.0f, A3 = 5.0f / 112.0f;
    const float A4 = 35.0f / 1152.0f, A5 = 63.0f / 2816.0f, A6 = 231.0f / 13312.0f;
    float y = mn(x2, 0.81f);
    return 1.0f + y * (A1 + y * (A2 + y * (A3 + y * (A4 + y * (A5 + y * (A6 / (1.0f - y)))))));
}

// transverse arc length of chord c on a circle of curvature k
__device__ __forceinline__ float arc(float c, float k)
{
    float x = (0.5f * k) * c;
    return c * asinx(x * x);
}

struct ModF {
    float cx, cy, cz, ux, uy, uz, vx, vy, vz, g, rl;
    int barrel, is2s;
    float wx, wy, wz;   // sensor normal (half-precision hit storage)
};

// Half-precision hit storage (the paper's outlook, Sec. 4): a hit is kept as
// its in-plane coordinates in its module's frame, relative to the module
// centre, each rounded to binary16 (nearest even), with its per-event index;
// the stages see the FP32 position rebuilt from them.  Fixed FP32 order.
__device__ __forceinline__ uint2 half_hit(const ModF &m, float x, float y, float z, int32_t idx)
{
    float dx = x - m.cx, dy = y - m.cy, dz = z - m.cz;
    float u = ((dx * m.ux) + (dy * m.uy)) + (dz * m.uz);
    float v = ((dx * m.vx) + (dy * m.vy)) + (dz * m.vz);
    const uint32_t hu = __builtin_bit_cast(uint16_t, (_Float16)u);
    const uint32_t hv = __builtin_bit_cast(uint16_t, (_Float16)v);
    return make_uint2(hu | (hv << 16), (uint32_t)idx);
}

// the FP32 position of grouped hit h on sensor `sensor` of module m (and its
// per-event index in w), from either storage
__device__ __forceinline__ float4 stored_hit(const EvDev &E, const ModF &m, uint32_t h, int sensor)
{
    if (!E.half16) return E.hsort[h];
    const uint2 r = E.hsort_h[h];
    const float u = (float)__builtin_bit_cast(_Float16, (uint16_t)(r.x & 0xffffu));
    const float v = (float)__builtin_bit_cast(_Float16, (uint16_t)(r.x >> 16));
    const float w = (sensor ? 0.5f : -0.5f) * m.g;
    return make_float4(((m.cx + (u * m.ux)) + (v * m.vx)) + (w * m.wx),
                       ((m.cy + (u * m.uy)) + (v * m.vy)) + (w * m.wy),
                       ((m.cz + (u * m.uz)) + (v * m.vz)) + (w * m.wz), __int_as_float((int32_t)r.y));
}

struct MdOut {
    float r, a, ca, bend, sv;
};

// radius of the lower hit and the sine / cosine of the threshold track's
// angle to the radius there
__device__ __forceinline__ void md_anchor(const Consts &K, float xL, float yL, MdOut &o)
{
    o.r = sqrtf((xL * xL) + (yL * yL));
    o.a = mn(o.r * K.kh, 0.999f);
    o.ca = sqrtf(1.0f - (o.a * o.a));
}

// Mini-doublet (stub) window for lower hit L and upper hit U of a module.
__device__ __forceinline__ bool md_accept(const Consts &K, const ModF &m, float xL, float yL,
                                          float zL, float xU, float yU, float zU, MdOut &o)
{
    float uL = (((xL - m.cx) * m.ux) + ((yL - m.cy) * m.uy)) + ((zL - m.cz) * m.uz);
    float vL = (((xL - m.cx) * m.vx) + ((yL - m.cy) * m.vy)) + ((zL - m.cz) * m.vz);
    float uU = (((xU - m.cx) * m.ux) + ((yU - m.cy) * m.uy)) + ((zU - m.cz) * m.uz);
    float vU = (((xU - m.cx) * m.vx) + ((yU - m.cy) * m.vy)) + ((zU - m.cz) * m.vz);
    float du = uU - uL;
    float dv = vU - vL;
    md_anchor(K, xL, yL, o);
    const float rL = o.r, a = o.a, ca = o.ca;
    float g = m.g;
    float hi, lo, zc, hz, sv;
    if (m.barrel) {
        // bend along u over the gap: g tan(psi +- alpha)
        float ta = a / ca;
        float tp = uL / m.rl;
        hi = g * ((tp + ta) / (1.0f - (tp * ta)));
        lo = g * ((tp - ta) / (1.0f + (tp * ta)));
        float dxy = sqrtf((du * du) + (g * g));
        zc = dxy * (zL / rL);
        hz = (dxy * (K.z0max / rL)) + K.tolv;
        sv = 0.0f;
    } else {
        // transverse step between the sensors, precise component sin(delta +- alpha)
        float sz = fabsf(zL);
        float Dlo = g * (rL / (sz + K.z0max));
        float Dhi = g * ((rL * asinx(a * a)) / (sz - K.z0max));
        float sp = uL / rL;
        float cp = ((xL * m.vx) + (yL * m.vy)) / rL;
        float Sp = (sp * ca) + (cp * a);
        float Sm = (sp * ca) - (cp * a);
        hi = mx(Dlo * Sp, Dhi * Sp);
        lo = mn(Dlo * Sm, Dhi * Sm);
        // the step's coarse (radial) component lies between Dlo cp and Dhi cp
        zc = (0.5f * (Dlo + Dhi)) * cp;
        hz = ((0.5f * (Dhi - Dlo)) * cp) + K.tolv;
        sv = sp;
    }
    float c0 = 0.5f * (hi + lo);
    float h0 = (0.5f * (hi - lo)) + K.tolu;
    o.bend = (du - c0) / h0;
    o.sv = sv;
    return (fabsf(du - c0) <= K.w * h0) && (fabsf(dv - zc) <= K.w * hz);
}

// A mini-doublet as the later stages see it (anchor = lower hit).
struct MdV {
    float x, y, z, r, a, ca, dx, dy, dn, sv, ir, svr;
    int barrel;
};

// the extra MD fields the learned scorer reads
struct MdX {
    float bend;
    int is2s;
};

__device__ __forceinline__ MdV load_md(const EvDev &E, int32_t i)
{
    MdV v;
    const float4 p0 = E.md_p0[i], p1 = E.md_p1[i], p2 = E.md_p2[i];
    v.x = p0.x; v.y = p0.y; v.z = p0.z; v.r = p0.w;
    v.a = p1.x; v.ca = p1.y; v.ir = p1.z; v.svr = p1.w;
    v.dx = p2.x; v.dy = p2.y; v.dn = p2.z; v.sv = p2.w;
    v.barrel = E.md_bar[i] & 1;
    return v;
}

__device__ __forceinline__ float tri_curv(const MdV &A, const MdV &B, const MdV &C)
{
    float xab = B.x - A.x, yab = B.y - A.y;
    float xbc = C.x - B.x, ybc = C.y - B.y;
    float xac = C.x - A.x, yac = C.y - A.y;
    float lab = sqrtf((xab * xab) + (yab * yab));
    float lbc = sqrtf((xbc * xbc) + (ybc * ybc));
    float lac = sqrtf((xac * xac) + (yac * yac));
    float crs = (xab * yac) - (yab * xac);
    return (2.0f * crs) / ((lab * lbc) * lac);
}

// Segment I -> O: azimuthal window (S2), pointing along the prompt circle
// (S1), relative angle of each barrel MD direction to the chord (S3).  The
// decision is the AND of the three cuts, so it is split in three calls that
// can run at different times, cheapest and most selective first:
// seg_window (S2, about a third of the pairs pass it), seg_angle (S3) and
// seg_point (S1).  They compute their shared terms by the same FP32
// operations, so together they give the single test's result.
// The azimuth window S2 decides exactly as `-(dot / rr) <= 0 && |crs / rr| <=
// B` would, but divides only when the division-free tests cannot decide:
//  * dot >= 0 implies -(dot / rr) <= 0 (rr > 0);
//  * with P = fl(B rr) a normal positive float, |crs| < fl(P (1 - 2^-20))
//    implies |crs| / rr < B, and |crs| > fl(P (1 + 2^-20)) implies
//    |crs| / rr > B (1 + 13 2^-24), i.e. above the float after B: the margin
//    2^-20 exceeds the three FP32 roundings (2^-24 each) between the two
//    forms, and rounding is monotone, so fl(|crs| / rr) falls on the same
//    side of B.  NaN and infinities take the exact path or agree with it.
// The per-MD terms 1 / r, |sv| / r and the S3 bound w (tol_u / |d|) come
// precomputed from the MD stage, rounded by the same FP32 operations.
__device__ __forceinline__ bool seg_window(const Consts &K, float xi, float yi, float ri, float ai,
                                           float cai, float iri, float svri, const float4 &p0,
                                           const float4 &p1)
{
    float rr = ri * p0.w;
    float crs = (xi * p0.y) - (yi * p0.x);
    float dot = (xi * p0.x) + (yi * p0.y);
    float sphi = (p1.x * cai) - (ai * p1.y);
    float tphi = (K.tolu * (iri + p1.z)) + (K.tolv * (svri + p1.w));
    float B = K.w * (sphi + tphi);
    bool c_ok = (dot >= 0.0f) || (-(dot / rr) <= 0.0f);
    float X = fabsf(crs), P = B * rr;
    bool s_ok;
    const bool p_ok = P >= 0x1p-100f;              // normal, far from underflow
    if (p_ok && X < P * 0x1.ffffep-1f)             // 1 - 2^-20
        s_ok = true;
    else if (p_ok && X > P * 0x1.00001p+0f)        // 1 + 2^-20
        s_ok = false;
    else
        s_ok = fabsf(crs / rr) <= B;
    return c_ok && s_ok;
}

// the inner MD as seg_angle and seg_point read it: anchor (x, y, z, r),
// direction (dx, dy, |d|, S3 bound), barrel flag
struct SegIn {
    float4 p, d;
    int barrel;
};

// S3: relative angle of each barrel MD's direction to the chord (about a
// fifth of the window survivors pass)
__device__ __forceinline__ bool seg_angle(const SegIn &I, const EvDev &E, int32_t o)
{
    const int ob = E.md_bar[o] & 1;
    if (!I.barrel && !ob) return true;
    const float4 p0 = E.md_p0[o];
    const float xi = I.p.x, yi = I.p.y, ri = I.p.w;
    float rr = ri * p0.w;
    float crs = (xi * p0.y) - (yi * p0.x);
    float S = crs / rr;
    float qx = p0.x - xi, qy = p0.y - yi;
    float ql = sqrtf((qx * qx) + (qy * qy));
    if (I.barrel) {
        float sa = ((I.d.x * qy) - (I.d.y * qx)) / (I.d.z * ql);
        if (!(fabsf(sa - S) <= I.d.w)) return false;
    }
    if (ob) {
        const float4 p2 = E.md_p2[o];
        float sb = ((qx * p2.y) - (qy * p2.x)) / (ql * p2.z);
        if (!(fabsf(sb - S) <= E.md_atol[o])) return false;
    }
    return true;
}

// S1: pointing of the r-z line along the prompt circle through both anchors
__device__ __forceinline__ bool seg_point(const Consts &K, const SegIn &I, const EvDev &E, int32_t o)
{
    const float4 p0 = E.md_p0[o];
    const int ob = E.md_bar[o] & 1;
    const float xi = I.p.x, yi = I.p.y, zi = I.p.z, ri = I.p.w;
    float rr = ri * p0.w;
    float crs = (xi * p0.y) - (yi * p0.x);
    float qx = p0.x - xi, qy = p0.y - yi;
    float ql = sqrtf((qx * qx) + (qy * qy));
    float kO = (2.0f * crs) / (rr * ql);
    float si = arc(ri, kO);
    float so = arc(p0.w, kO);
    float ds = so - si;
    float z0 = ((zi * so) - (p0.z * si)) / ds;
    float sl = (p0.z - zi) / ds;
    float szi = I.barrel ? K.sigv : (fabsf(sl) * K.sigv);
    float szo = ob ? K.sigv : (fabsf(sl) * K.sigv);
    float tolz = K.nsig * (((so * szi) + (si * szo)) / ds);
    return fabsf(z0) <= K.w * (K.z0max + tolz);
}

// S3 bound of an MD with direction length dn (the MD stage stores it)
__device__ __forceinline__ float seg_angle_bound(const Consts &K, float dn)
{
    return K.w * (K.tolu / dn);
}

// variance of an anchor along the track normal
__device__ __forceinline__ float perp_var(const Consts &K, const MdV &P, float hk)
{
    float su2 = K.sigu * K.sigu;
    float t = P.sv + (hk * P.r);
    float e = K.sigv * t;
    return P.barrel ? su2 : (su2 + (e * e));
}

// Triplet A-B-C: curvature bound (T1), beam-line circle (T2), r-z line (T3).
__device__ __forceinline__ bool t3_accept(const Consts &K, const MdV &A, const MdV &B,
                                          const MdV &C, float &k_out)
{
    float xab = B.x - A.x, yab = B.y - A.y;
    float xbc = C.x - B.x, ybc = C.y - B.y;
    float xac = C.x - A.x, yac = C.y - A.y;
    float lab = sqrtf((xab * xab) + (yab * yab));
    float lbc = sqrtf((xbc * xbc) + (ybc * ybc));
    float lac = sqrtf((xac * xac) + (yac * yac));
    float crs = (xab * yac) - (yab * xac);
    float k = (2.0f * crs) / ((lab * lbc) * lac);
    k_out = k;
    float l2 = lac * lac;
    float hk = 0.5f * k;
    float e2 = mx(mx(perp_var(K, A, hk), perp_var(K, B, hk)), perp_var(K, C, hk));
    float tk = (K.tolkc * sqrtf(e2)) / l2;
    if (!(fabsf(k) <= K.w * (K.klim + tk))) return false;
    float kO = (2.0f * ((A.x * C.y) - (A.y * C.x))) / ((A.r * C.r) * lac);
    if (!(fabsf(k - kO) <= K.w * (tk + ((2.0f * K.d0max) / (A.r * C.r))))) return false;
    float sab = arc(lab, k);
    float sbc = arc(lbc, k);
    float st = sab + sbc;
    float f = sab / st;
    float sl = (C.z - A.z) / st;
    float dz = B.z - (A.z + ((C.z - A.z) * f));
    float se = mx(fabsf(sl), 0.05f) * K.sigv;
    float sza = A.barrel ? K.sigv : se;
    float szb = B.barrel ? K.sigv : se;
    float szc = C.barrel ? K.sigv : se;
    float g1 = (1.0f - f) * sza;
    float g2 = f * szc;
    return fabsf(dz) <= K.w * (K.nsig * sqrtf(((szb * szb) + (g1 * g1)) + (g2 * g2)));
}

// signed distance of P from the circle through A, C, E
__device__ __forceinline__ float circ_res(float xa, float ya, float xc, float yc, float xe,
                                         float ye, float xp, float yp, float crs, float den)
{
    float Ax = xa - xp, Ay = ya - yp;
    float Cx = xc - xp, Cy = yc - yp;
    float Ex = xe - xp, Ey = ye - yp;
    float la = (Ax * Ax) + (Ay * Ay);
    float lc = (Cx * Cx) + (Cy * Cy);
    float le = (Ex * Ex) + (Ey * Ey);
    float det = ((Ax * ((Cy * le) - (lc * Ey))) - (Ay * ((Cx * le) - (lc * Ex)))) +
                (la * ((Cx * Ey) - (Cy * Ex)));
    float sd = (crs >= 0.0f) ? -det : det;
    return sd / den;
}

// Quintuplet P0..P4 from triplets (P0,P1,P2) and (P2,P3,P4): curvature
// agreement with the bridge circle (Q1), bridge curvature bound (Q2), r-phi
// chi2 of P1 and P3 (Q3), r-z chi2 of P1..P3 (Q4).  score = chi2 sum.
__device__ __forceinline__ bool t5_accept(const Consts &K, const MdV &A, const MdV &B,
                                          const MdV &C, const MdV &D, const MdV &Ee, float kin,
                                          float kout, float &score)
{
    float xac = C.x - A.x, yac = C.y - A.y;
    float xce = Ee.x - C.x, yce = Ee.y - C.y;
    float xae = Ee.x - A.x, yae = Ee.y - A.y;
    float lac = sqrtf((xac * xac) + (yac * yac));
    float lce = sqrtf((xce * xce) + (yce * yce));
    float lae = sqrtf((xae * xae) + (yae * yae));
    float crs = (xac * yae) - (yac * xae);
    float den = (lac * lce) * lae;
    float kbr = (2.0f * crs) / den;
    float hk = 0.5f * kbr;
    float v0 = perp_var(K, A, hk), v1 = perp_var(K, B, hk), v2 = perp_var(K, C, hk);
    float v3 = perp_var(K, D, hk), v4 = perp_var(K, Ee, hk);
    float ein = mx(mx(v0, v1), v2);
    float eout = mx(mx(v2, v3), v4);
    if (!(fabsf(kin - kbr) <= K.w * (((K.tolkc * sqrtf(ein)) / (lac * lac)) + K.epsak))) return false;
    if (!(fabsf(kout - kbr) <= K.w * (((K.tolkc * sqrtf(eout)) / (lce * lce)) + K.epsak))) return false;
    if (!(fabsf(kbr) <= K.w * K.klim)) return false;
    float resb = circ_res(A.x, A.y, C.x, C.y, Ee.x, Ee.y, B.x, B.y, crs, den);
    float resd = circ_res(A.x, A.y, C.x, C.y, Ee.x, Ee.y, D.x, D.y, crs, den);
    float xab = B.x - A.x, yab = B.y - A.y;
    float xbc = C.x - B.x, ybc = C.y - B.y;
    float xcd = D.x - C.x, ycd = D.y - C.y;
    float xde = Ee.x - D.x, yde = Ee.y - D.y;
    float s1 = arc(sqrtf((xab * xab) + (yab * yab)), kbr);
    float s2 = arc(sqrtf((xbc * xbc) + (ybc * ybc)), kbr);
    float s3 = arc(sqrtf((xcd * xcd) + (ycd * ycd)), kbr);
    float s4 = arc(sqrtf((xde * xde) + (yde * yde)), kbr);
    float S1 = s1, S2 = S1 + s2, S3 = S2 + s3, S4 = S3 + s4;
    float Lab = ((S1 - S2) * (S1 - S4)) / (S2 * S4);
    float Lcb = (S1 * (S1 - S4)) / (S2 * (S2 - S4));
    float Leb = (S1 * (S1 - S2)) / (S4 * (S4 - S2));
    float Lad = ((S3 - S2) * (S3 - S4)) / (S2 * S4);
    float Lcd = (S3 * (S3 - S4)) / (S2 * (S2 - S4));
    float Led = (S3 * (S3 - S2)) / (S4 * (S4 - S2));
    float Vb = (v1 + (((Lab * Lab) * v0) + ((Lcb * Lcb) * v2))) + ((Leb * Leb) * v4);
    float Vd = (v3 + (((Lad * Lad) * v0) + ((Lcd * Lcd) * v2))) + ((Led * Led) * v4);
    float chi2p = ((resb * resb) / Vb) + ((resd * resd) / Vd);
    if (!(chi2p <= K.w2 * K.xrphi)) return false;
    float sl = (Ee.z - A.z) / S4;
    float se = mx(fabsf(sl), 0.05f) * K.sigv;
    float sza = A.barrel ? K.sigv : se;
    float sze = Ee.barrel ? K.sigv : se;
    float szb = B.barrel ? K.sigv : se;
    float szc = C.barrel ? K.sigv : se;
    float szd = D.barrel ? K.sigv : se;
    float tb, tc, td;
    {
        float f = S1 / S4;
        float dz = B.z - (A.z + (sl * S1));
        float g1 = (1.0f - f) * sza, g2 = f * sze;
        float V = ((szb * szb) + (g1 * g1)) + (g2 * g2);
        tb = (dz * dz) / V;
    }
    {
        float f = S2 / S4;
        float dz = C.z - (A.z + (sl * S2));
        float g1 = (1.0f - f) * sza, g2 = f * sze;
        float V = ((szc * szc) + (g1 * g1)) + (g2 * g2);
        tc = (dz * dz) / V;
    }
    {
        float f = S3 / S4;
        float dz = D.z - (A.z + (sl * S3));
        float g1 = (1.0f - f) * sza, g2 = f * sze;
        float V = ((szd * szd) + (g1 * g1)) + (g2 * g2);
        td = (dz * dz) / V;
    }
    float chi2z = (tb + tc) + td;
    if (!(chi2z <= K.w2 * K.xrz)) return false;
    score = chi2p + chi2z;
    return true;
}

// ---------------------------------------------------------------- pixel objects
// Direction of an object without transcendental functions: the circle
// through the beam line and points A (inner) and E (outer) has its tangent at
// the beam line along A/|A|^2 - E/|E|^2 (the image of the circle under
// inversion about the origin is the line through the images of A and E).
__device__ __forceinline__ void dir2(float xa, float ya, float xe, float ye, float &tx, float &ty)
{
    float ra2 = (xa * xa) + (ya * ya);
    float re2 = (xe * xe) + (ye * ye);
    tx = (xa / ra2) - (xe / re2);
    ty = (ya / ra2) - (ye / re2);
}

// pLS direction: tangent from its first and last pixel hits, polar slope of
// their chord
__device__ __forceinline__ float4 pls_dir(float x1, float y1, float z1, float x4, float y4, float z4)
{
    float tx, ty;
    dir2(x1, y1, x4, y4, tx, ty);
    float dx = x4 - x1, dy = y4 - y1;
    return make_float4(tx, ty, (z4 - z1) / sqrtf((dx * dx) + (dy * dy)), 0.0f);
}

// outer object direction from its first and last anchors and curvature k:
// polar slope = dz over the arc length
__device__ __forceinline__ float4 obj_dir(const MdV &A, const MdV &E, float k)
{
    float tx, ty;
    dir2(A.x, A.y, E.x, E.y, tx, ty);
    float dx = E.x - A.x, dy = E.y - A.y;
    return make_float4(tx, ty, (E.z - A.z) / arc(sqrtf((dx * dx) + (dy * dy)), k), 0.0f);
}

// bridge curvature of a quintuplet from its anchors A, C, E
__device__ __forceinline__ float bridge_curv(const MdV &A, const MdV &C, const MdV &E)
{
    float xac = C.x - A.x, yac = C.y - A.y;
    float xce = E.x - C.x, yce = E.y - C.y;
    float xae = E.x - A.x, yae = E.y - A.y;
    float lac = sqrtf((xac * xac) + (yac * yac));
    float lce = sqrtf((xce * xce) + (yce * yce));
    float lae = sqrtf((xae * xae) + (yae * yae));
    float crs = (xac * yae) - (yac * xae);
    return (2.0f * crs) / ((lac * lce) * lae);
}

// azimuthal and polar separation of two directions: cos-term, sin^2(dphi),
// (dcot)^2 / (1 + (c1^2 + c2^2) / 2)
__device__ __forceinline__ void dir_sep(const float4 &a, const float4 &b, float &dot, float &sp2,
                                        float &se2)
{
    dot = (a.x * b.x) + (a.y * b.y);
    float crs = (a.x * b.y) - (a.y * b.x);
    float nn = ((a.x * a.x) + (a.y * a.y)) * ((b.x * b.x) + (b.y * b.y));
    sp2 = (crs * crs) / nn;
    float dc = a.z - b.z;
    se2 = (dc * dc) / (1.0f + (0.5f * ((a.z * a.z) + (b.z * b.z))));
}

// linking window: same hemisphere, sin^2(dphi) and polar term within wl2
__device__ __forceinline__ bool link_window(const float4 &a, const float4 &b, float wl2)
{
    float dot, sp2, se2;
    dir_sep(a, b, dot, sp2, se2);
    return (-dot <= 0.0f) && (sp2 <= wl2) && (se2 <= wl2);
}

// cross-cleaning: same hemisphere and sin^2(dphi) + polar term within dr2
__device__ __forceinline__ bool close_dir(const float4 &a, const float4 &b, float dr2)
{
    float dot, sp2, se2;
    dir_sep(a, b, dot, sp2, se2);
    return (-dot <= 0.0f) && ((sp2 + se2) <= dr2);
}

// a point of a linked chain: pixel hit (kind 0) or anchor (1 barrel, 2 endcap)
struct LPt {
    float x, y, z, sv, r;
    int kind;
};

__device__ __forceinline__ LPt lpt_md(const MdV &m)
{
    LPt p;
    p.x = m.x; p.y = m.y; p.z = m.z; p.sv = m.sv; p.r = m.r;
    p.kind = m.barrel ? 1 : 2;
    return p;
}

__device__ __forceinline__ LPt lpt_px(float x, float y, float z)
{
    LPt p;
    p.x = x; p.y = y; p.z = z; p.sv = 0.0f; p.r = 0.0f; p.kind = 0;
    return p;
}

// Link chi2 of a chain of N points (pLS hits then anchors): circle through
// points 0, IC and N-1; r-phi chi2 of the others with Lagrange-propagated
// node variances; r-z chi2 of points 1..N-2 about the line in arc length
// through 0 and N-1; both sums taken in point order.  Cuts against
// w^2 x2p and w^2 x2z; score = chi2_rphi + chi2_rz.
template <int N, int IC>
__device__ __forceinline__ bool link_accept(const Consts &K, const LPt *p, float sig2p,
                                            float sigz, float x2p, float x2z, float &score)
{
    const float xa = p[0].x, ya = p[0].y, za = p[0].z;
    const float xc = p[IC].x, yc = p[IC].y;
    const float xe = p[N - 1].x, ye = p[N - 1].y, ze = p[N - 1].z;
    float xac = xc - xa, yac = yc - ya;
    float xce = xe - xc, yce = ye - yc;
    float xae = xe - xa, yae = ye - ya;
    float lac = sqrtf((xac * xac) + (yac * yac));
    float lce = sqrtf((xce * xce) + (yce * yce));
    float lae = sqrtf((xae * xae) + (yae * yae));
    float crs = (xac * yae) - (yac * xae);
    float den = (lac * lce) * lae;
    float k = (2.0f * crs) / den;
    float hk = 0.5f * k;
    float s[N], vp[N];
    s[0] = 0.0f;
#pragma unroll
    for (int j = 1; j < N; ++j) {
        float dx = p[j].x - p[j - 1].x, dy = p[j].y - p[j - 1].y;
        s[j] = s[j - 1] + arc(sqrtf((dx * dx) + (dy * dy)), k);
    }
    const float su2 = K.sigu * K.sigu;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        if (p[j].kind == 0) {
            vp[j] = sig2p;
        } else {
            float e = K.sigv * (p[j].sv + (hk * p[j].r));
            vp[j] = p[j].kind == 1 ? su2 : (su2 + (e * e));
        }
    }
    const float sc = s[IC], se = s[N - 1];
    float chi2p = 0.0f;
#pragma unroll
    for (int j = 1; j < N - 1; ++j) {
        if (j == IC) continue;
        float res = circ_res(xa, ya, xc, yc, xe, ye, p[j].x, p[j].y, crs, den);
        float sj = s[j];
        float L0 = ((sj - sc) * (sj - se)) / (sc * se);
        float Lc = (sj * (sj - se)) / (sc * (sc - se));
        float Le = (sj * (sj - sc)) / (se * (se - sc));
        float V = (vp[j] + (((L0 * L0) * vp[0]) + ((Lc * Lc) * vp[IC]))) + ((Le * Le) * vp[N - 1]);
        chi2p = chi2p + ((res * res) / V);
    }
    float sl = (ze - za) / se;
    float sev = mx(fabsf(sl), 0.05f) * K.sigv;
    float sz0 = p[0].kind == 0 ? sigz : p[0].kind == 1 ? K.sigv : sev;
    float sze = p[N - 1].kind == 0 ? sigz : p[N - 1].kind == 1 ? K.sigv : sev;
    float chi2z = 0.0f;
#pragma unroll
    for (int j = 1; j < N - 1; ++j) {
        float szj = p[j].kind == 0 ? sigz : p[j].kind == 1 ? K.sigv : sev;
        float f = s[j] / se;
        float dz = p[j].z - (za + (sl * s[j]));
        float g1 = (1.0f - f) * sz0;
        float g2 = f * sze;
        float V = ((szj * szj) + (g1 * g1)) + (g2 * g2);
        chi2z = chi2z + ((dz * dz) / V);
    }
    score = chi2p + chi2z;
    return (chi2p <= K.w2 * x2p) && (chi2z <= K.w2 * x2z);
}

// Every triplet quantity of t3_accept, without early exits, and the 40
// features of the learned scorer (22 used, the rest zero; same operation
// order as t3_accept for the shared quantities): per MD r/100, z/100, bend
// pull, endcap flag, 2S flag; curvature over kappa_max; each cut's left-hand
// side over its limit (|k|, signed k - k_origin, signed r-z residual); r-z
// slope; chord/100; impact-parameter estimate (k - k_origin) r_a r_c / 2.
__device__ __forceinline__ void t3_features(const Consts &K, const MdV *P, const MdX *X, float *f)
{
    const MdV &A = P[0], &B = P[1], &C = P[2];
    float xab = B.x - A.x, yab = B.y - A.y;
    float xbc = C.x - B.x, ybc = C.y - B.y;
    float xac = C.x - A.x, yac = C.y - A.y;
    float lab = sqrtf((xab * xab) + (yab * yab));
    float lbc = sqrtf((xbc * xbc) + (ybc * ybc));
    float lac = sqrtf((xac * xac) + (yac * yac));
    float crs = (xab * yac) - (yab * xac);
    float k = (2.0f * crs) / ((lab * lbc) * lac);
    float l2 = lac * lac;
    float hk = 0.5f * k;
    float e2 = mx(mx(perp_var(K, A, hk), perp_var(K, B, hk)), perp_var(K, C, hk));
    float tk = (K.tolkc * sqrtf(e2)) / l2;
    float rhs0 = K.w * (K.klim + tk);
    float kO = (2.0f * ((A.x * C.y) - (A.y * C.x))) / ((A.r * C.r) * lac);
    float rhs1 = K.w * (tk + ((2.0f * K.d0max) / (A.r * C.r)));
    float sab = arc(lab, k);
    float sbc = arc(lbc, k);
    float st = sab + sbc;
    float fr = sab / st;
    float sl = (C.z - A.z) / st;
    float dz = B.z - (A.z + ((C.z - A.z) * fr));
    float se = mx(fabsf(sl), 0.05f) * K.sigv;
    float sza = A.barrel ? K.sigv : se;
    float szb = B.barrel ? K.sigv : se;
    float szc = C.barrel ? K.sigv : se;
    float g1 = (1.0f - fr) * sza;
    float g2 = fr * szc;
    float rhs2 = K.w * (K.nsig * sqrtf(((szb * szb) + (g1 * g1)) + (g2 * g2)));
#pragma unroll
    for (int j = 0; j < 40; ++j) f[j] = 0.0f;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        f[5 * j + 0] = P[j].r * 0.01f;
        f[5 * j + 1] = P[j].z * 0.01f;
        f[5 * j + 2] = X[j].bend;
        f[5 * j + 3] = P[j].barrel ? 0.0f : 1.0f;
        f[5 * j + 4] = X[j].is2s ? 1.0f : 0.0f;
    }
    f[15] = k / K.kmax;
    f[16] = fabsf(k) / rhs0;
    f[17] = (k - kO) / rhs1;
    f[18] = dz / rhs2;
    f[19] = sl;
    f[20] = lac * 0.01f;
    f[21] = ((k - kO) * (A.r * C.r)) * 0.5f;
}

// Every quintuplet quantity of t5_accept, without early exits, and the 40
// features of the learned scorer (same operation order as t5_accept for the
// shared quantities): per MD r/100, z/100, bend pull, endcap flag, 2S flag;
// curvatures over kappa_max; chi2/(1+chi2) for r-phi and r-z; r-phi pulls of
// the 2nd and 4th anchors; r-z pulls of the 2nd..4th; curvature agreement
// over its tolerance (inner, outer); r-z slope; lever arm/100; transverse
// impact parameter estimate.
__device__ __forceinline__ void t5_features(const Consts &K, const MdV *P, const MdX *X, float kin,
                                            float kout, float *f)
{
    const MdV &A = P[0], &B = P[1], &C = P[2], &D = P[3], &Ee = P[4];
    float xac = C.x - A.x, yac = C.y - A.y;
    float xce = Ee.x - C.x, yce = Ee.y - C.y;
    float xae = Ee.x - A.x, yae = Ee.y - A.y;
    float lac = sqrtf((xac * xac) + (yac * yac));
    float lce = sqrtf((xce * xce) + (yce * yce));
    float lae = sqrtf((xae * xae) + (yae * yae));
    float crs = (xac * yae) - (yac * xae);
    float den = (lac * lce) * lae;
    float kbr = (2.0f * crs) / den;
    float hk = 0.5f * kbr;
    float v0 = perp_var(K, A, hk), v1 = perp_var(K, B, hk), v2 = perp_var(K, C, hk);
    float v3 = perp_var(K, D, hk), v4 = perp_var(K, Ee, hk);
    float ein = mx(mx(v0, v1), v2);
    float eout = mx(mx(v2, v3), v4);
    float tin = ((K.tolkc * sqrtf(ein)) / (lac * lac)) + K.epsak;
    float tout = ((K.tolkc * sqrtf(eout)) / (lce * lce)) + K.epsak;
    float resb = circ_res(A.x, A.y, C.x, C.y, Ee.x, Ee.y, B.x, B.y, crs, den);
    float resd = circ_res(A.x, A.y, C.x, C.y, Ee.x, Ee.y, D.x, D.y, crs, den);
    float xab = B.x - A.x, yab = B.y - A.y;
    float xbc = C.x - B.x, ybc = C.y - B.y;
    float xcd = D.x - C.x, ycd = D.y - C.y;
    float xde = Ee.x - D.x, yde = Ee.y - D.y;
    float s1 = arc(sqrtf((xab * xab) + (yab * yab)), kbr);
    float s2 = arc(sqrtf((xbc * xbc) + (ybc * ybc)), kbr);
    float s3 = arc(sqrtf((xcd * xcd) + (ycd * ycd)), kbr);
    float s4 = arc(sqrtf((xde * xde) + (yde * yde)), kbr);
    float S1 = s1, S2 = S1 + s2, S3 = S2 + s3, S4 = S3 + s4;
    float Lab = ((S1 - S2) * (S1 - S4)) / (S2 * S4);
    float Lcb = (S1 * (S1 - S4)) / (S2 * (S2 - S4));
    float Leb = (S1 * (S1 - S2)) / (S4 * (S4 - S2));
    float Lad = ((S3 - S2) * (S3 - S4)) / (S2 * S4);
    float Lcd = (S3 * (S3 - S4)) / (S2 * (S2 - S4));
    float Led = (S3 * (S3 - S2)) / (S4 * (S4 - S2));
    float Vb = (v1 + (((Lab * Lab) * v0) + ((Lcb * Lcb) * v2))) + ((Leb * Leb) * v4);
    float Vd = (v3 + (((Lad * Lad) * v0) + ((Lcd * Lcd) * v2))) + ((Led * Led) * v4);
    float chi2p = ((resb * resb) / Vb) + ((resd * resd) / Vd);
    float sl = (Ee.z - A.z) / S4;
    float se = mx(fabsf(sl), 0.05f) * K.sigv;
    float sza = A.barrel ? K.sigv : se;
    float sze = Ee.barrel ? K.sigv : se;
    float Sj[3] = {S1, S2, S3};
    float zj[3] = {B.z, C.z, D.z};
    float szj[3] = {B.barrel ? K.sigv : se, C.barrel ? K.sigv : se, D.barrel ? K.sigv : se};
    float t[3], pull[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        float fr = Sj[j] / S4;
        float dz = zj[j] - (A.z + (sl * Sj[j]));
        float g1 = (1.0f - fr) * sza, g2 = fr * sze;
        float V = ((szj[j] * szj[j]) + (g1 * g1)) + (g2 * g2);
        t[j] = (dz * dz) / V;
        pull[j] = dz / sqrtf(V);
    }
    float chi2z = (t[0] + t[1]) + t[2];
    float kO = (2.0f * ((A.x * Ee.y) - (A.y * Ee.x))) / ((A.r * Ee.r) * lae);
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        f[5 * j + 0] = P[j].r * 0.01f;
        f[5 * j + 1] = P[j].z * 0.01f;
        f[5 * j + 2] = X[j].bend;
        f[5 * j + 3] = P[j].barrel ? 0.0f : 1.0f;
        f[5 * j + 4] = X[j].is2s ? 1.0f : 0.0f;
    }
    f[25] = kin / K.kmax;
    f[26] = kout / K.kmax;
    f[27] = kbr / K.kmax;
    f[28] = chi2p / (1.0f + chi2p);
    f[29] = chi2z / (1.0f + chi2z);
    f[30] = resb / sqrtf(Vb);
    f[31] = resd / sqrtf(Vd);
    f[32] = pull[0];
    f[33] = pull[1];
    f[34] = pull[2];
    f[35] = (kin - kbr) / tin;
    f[36] = (kout - kbr) / tout;
    f[37] = sl;
    f[38] = lae * 0.01f;
    f[39] = ((kbr - kO) * (A.r * Ee.r)) * 0.5f;
}

}  // namespace lst
