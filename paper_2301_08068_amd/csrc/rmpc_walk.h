// rmpc_walk.h -- device-side pieces of the exact ray walk shared by the dense-grid kernels
// (raycast.hip) and the sparse block-map kernels (sparse.hip): float32 crossing parameters with
// float64 decisions inside a guard band, segment boundaries, entry voxels of coarse elements,
// the per-ray obstacle policy, and launch helpers.  gfx950 only.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "rmpc_device.h"
#include "rmpc_kernels.h"

namespace rmpc {

constexpr float kInf = __builtin_huge_valf();
// Voxel units between a segment boundary t and any face crossing: kSegMargin + kSegMarginRel * t.
// A float32 crossing parameter is within 1.8e-7 T of its value and t_hi = float32(t) within
// 6e-8 t, so no float32 end test can land on the wrong side; below 0.025 for any t up to the
// diagonal of a 4096^3 grid, so one crossing excludes at most one of the 0.05-spaced candidates.
constexpr double kSegMargin = 1e-3;
constexpr double kSegMarginRel = 1e-6;

// Requires x in a vector register at this point (emits no instruction): the per-step masks of
// a round are folded into integer bit masks step by step instead of being carried as 64-bit
// comparison masks in scalar registers until the end of the round.
template <class T>
__device__ __forceinline__ void in_vgpr(T &x)
{
    asm volatile("" : "+v"(x));
}

// Smallest float above x >= 0 (x itself if +inf): t > x  <=>  t >= next_up(x).
__device__ __forceinline__ float next_up(float x)
{
    return x < kInf ? __int_as_float(__float_as_int(x) + 1) : x;
}

// Float64 crossing parameter of the next face along one axis (r != 0) from voxel coordinate v.
__device__ __forceinline__ double cross64(int v, float g, float r)
{
    const double B = r > 0.0f ? (double)(v + 1) : (double)v;
    return (B - (double)g) / (double)r;
}

// Float64 parameter at which the ray entered voxel coordinate v along one axis (r != 0).
__device__ __forceinline__ double entry64(int v, float g, float r)
{
    const double B = r > 0.0f ? (double)v : (double)(v + 1);
    return (B - (double)g) / (double)r;
}


// Segment boundary of a ray near t_nom: the first of 16 candidates t = t_nom + 0.05 c (voxel
// units) whose distance to every face crossing of the ray is at least the margin.  Within 0.8
// voxel units each axis crosses at most two faces, so at most six candidates are excluded and
// the search cannot fail for real inputs; `ok` is false otherwise.  Returns the voxel there.
__device__ __forceinline__ double seg_boundary(double t_nom, float gx, float gy, float gz, float rx,
                                               float ry, float rz, int &vx, int &vy, int &vz, bool &ok)
{
    ok = false;
    double t = t_nom;
    for (int c = 0; c < 16 && !ok; ++c) {
        t = t_nom + 0.05 * c;
        vx = (int)floor((double)gx + t * (double)rx);
        vy = (int)floor((double)gy + t * (double)ry);
        vz = (int)floor((double)gz + t * (double)rz);
        const double mg = kSegMargin + kSegMarginRel * t;
        bool good = true;
        if (rx != 0.0f) good = good && cross64(vx, gx, rx) - t >= mg && t - entry64(vx, gx, rx) >= mg;
        if (ry != 0.0f) good = good && cross64(vy, gy, ry) - t >= mg && t - entry64(vy, gy, ry) >= mg;
        if (rz != 0.0f) good = good && cross64(vz, gz, rz) - t >= mg && t - entry64(vz, gz, rz) >= mg;
        ok = good;
    }
    return t;
}

// Float64 parameter of the face at integer coordinate B along one axis (r != 0).
__device__ __forceinline__ double face64(int B, float g, float r)
{
    return ((double)B - (double)g) / (double)r;
}

// The ray in the forms the walk uses.  Along each axis the walk only moves toward larger
// s*coordinate (s = sign of r), so faces are kept as s*B: a step adds the level's edge, and
// the float32 crossing parameter (s*B - s*g) * |1/r| has the same bits as (B - g) * (1/r).
struct RayF {
    float gx, gy, gz;                 // start, grid units
    float rx, ry, rz;                 // direction
    float gsx, gsy, gsz;              // s*g
    float arx, ary, arz;              // |1/r|, +inf for r = 0
};

__device__ __forceinline__ RayF make_ray(const RayArgs &A, float rx, float ry, float rz)
{
    RayF R;
    R.gx = A.g[0]; R.gy = A.g[1]; R.gz = A.g[2];
    R.rx = rx; R.ry = ry; R.rz = rz;
    R.gsx = rx > 0.0f ? R.gx : -R.gx;
    R.gsy = ry > 0.0f ? R.gy : -R.gy;
    R.gsz = rz > 0.0f ? R.gz : -R.gz;
    R.arx = rx != 0.0f ? fabsf(1.0f / rx) : kInf;
    R.ary = ry != 0.0f ? fabsf(1.0f / ry) : kInf;
    R.arz = rz != 0.0f ? fabsf(1.0f / rz) : kInf;
    return R;
}

// Does face F of axis b come before the crossing of face Ba of axis a in the merged crossing
// order (a smaller parameter, or an equal one on a lower axis)?  Float32 decides outside the
// guard band, float64 inside it.
__device__ __forceinline__ bool crossed_first(int F, float gb, float rb, float irb, int b, float T32, int Ba,
                                              float ga, float ra, int a, bool &tie)
{
    const float tf = ((float)F - gb) * irb;
    const float band = 2e-5f + 1e-6f * fmaxf(fabsf(tf), T32);
    if (tf < T32 - band) return true;
    if (tf > T32 + band) return false;
    const double f64 = face64(F, gb, rb), t64 = face64(Ba, ga, ra);
    tie = tie || fabs(f64 - t64) < 1e-5;
    return f64 < t64 || (f64 == t64 && b < a);
}

// Coordinate along axis b (rb != 0) of the voxel the walk is in right after crossing face Ba
// of axis a at float32 parameter T32, known to lie in [lo, hi] (the entered element's extent,
// cut at the start voxel): the float32 estimate floor(g + T r), confirmed on the face behind
// it and the face ahead of it, except on the bounds of [lo, hi].
__device__ __forceinline__ int entry_coord(int lo, int hi, float gb, float rb, float irb, int b, float T32, int Ba,
                                           float ga, float ra, int a, bool &tie)
{
    const float y = fmaf(T32, rb, gb);
    int c = (int)floorf(y);
    // y is within 1.8e-7 |T r| + 1.2e-7 |y| of g + T r (T32 carries three roundings, the fma
    // one): away from a face by twice that, floor(y) is the answer; near a face the two
    // bounding faces are checked in the crossing order
    const float fr = y - floorf(y);
    const float tol = 4e-7f * fabsf(T32 * rb) + 3e-7f * fabsf(y) + 1e-6f;
    if (fr > tol && fr < 1.0f - tol && c >= lo && c <= hi) return c;
    c = min(max(c, lo), hi);
    const bool up = rb > 0.0f;
    const int f_in = up ? c : c + 1;              // face crossed into voxel c
    const int f_out = up ? c + 1 : c;             // face out of voxel c, ahead
    const bool chk_in = up ? c > lo : c < hi;     // the cell's own face needs no check
    const bool chk_out = up ? c < hi : c > lo;
    if (chk_in && !crossed_first(f_in, gb, rb, irb, b, T32, Ba, ga, ra, a, tie))
        c += up ? -1 : 1;
    else if (chk_out && crossed_first(f_out, gb, rb, irb, b, T32, Ba, ga, ra, a, tie))
        c += up ? 1 : -1;
    return c;
}

// Voxel the walk is in right after entering element (cx, cy, cz) of level lg (a brick or a
// cell) across its face on axis a.
__device__ __forceinline__ void entry_voxel(const RayArgs &A, const RayF &R, int lg, int a, int cx, int cy, int cz,
                                           int &vx, int &vy, int &vz, bool &tie)
{
    const int E = 1 << lg;
    const float gx = R.gx, gy = R.gy, gz = R.gz, rx = R.rx, ry = R.ry, rz = R.rz;
    const int px = rx > 0.0f, py = ry > 0.0f, pz = rz > 0.0f;
    // 1/r with the bits of the walk's own reciprocal
    const float irx = px ? R.arx : -R.arx, iry = py ? R.ary : -R.ary, irz = pz ? R.arz : -R.arz;
    const int lx = cx * E, ly = cy * E, lz = cz * E;          // (coordinates may be negative)
    // the face crossed: the cell's low face when travelling up the axis, else its high face
    const int Ba = a == 0 ? (px ? lx : lx + E) : (a == 1 ? (py ? ly : ly + E) : (pz ? lz : lz + E));
    const float ga = a == 0 ? gx : (a == 1 ? gy : gz);
    const float ra = a == 0 ? rx : (a == 1 ? ry : rz);
    const float ira = a == 0 ? irx : (a == 1 ? iry : irz);
    const float T32 = ((float)Ba - ga) * ira;
    // along each other axis the walk never moves back past its start voxel, so a face at or
    // behind the start is no decision of the walk (a start on such a face is not a near-tie)
    const int x0 = A.v0[0], y0 = A.v0[1], z0 = A.v0[2];
    const int xlo = px ? max(lx, x0) : lx, xhi = px ? lx + E - 1 : min(lx + E - 1, x0);
    const int ylo = py ? max(ly, y0) : ly, yhi = py ? ly + E - 1 : min(ly + E - 1, y0);
    const int zlo = pz ? max(lz, z0) : lz, zhi = pz ? lz + E - 1 : min(lz + E - 1, z0);
    vx = a == 0 ? (px ? lx : lx + E - 1) : (rx != 0.0f ? entry_coord(xlo, xhi, gx, rx, irx, 0, T32, Ba, ga, ra, a, tie) : x0);
    vy = a == 1 ? (py ? ly : ly + E - 1) : (ry != 0.0f ? entry_coord(ylo, yhi, gy, ry, iry, 1, T32, Ba, ga, ra, a, tie) : y0);
    vz = a == 2 ? (pz ? lz : lz + E - 1) : (rz != 0.0f ? entry_coord(zlo, zhi, gz, rz, irz, 2, T32, Ba, ga, ra, a, tie) : z0);
}

// Entry j of an ordered ray list as one 16-byte load: direction in x, y, z, Halton index bits in w.
__device__ __forceinline__ float4 load_ray(const RayRec *rays, int j)
{
    return reinterpret_cast<const float4 *>(rays)[j];
}

// The obstacle policy of one hit ray (Sec. III-C, Eqs. 4-9), float32, folded into the
// rank-one form  A_i = a r r^T,  b_i = -a |r|^2 phi r  with
//   p = max(0, xdot . r)^2,  q = eta_damp p / (d/nu_damp + eps)        (|f_damp| / |r|)
//   sigma = q / (q|r| + c log(1 + exp(-2 c q|r|)))                      (s(f_damp) = -sigma r)
//   a = w_r(d) sigma^2,  phi = eta_rep exp(-d/nu_rep) + q,  w_r(d) = (1 - d/r)^2 on [0, r].
__device__ __forceinline__ void policy_accumulate(const PolicyF &P, float rx, float ry, float rz,
                                                  float d, Acc &acc)
{
    const float vr = P.vx * rx + P.vy * ry + P.vz * rz;
    const float pp = vr > 0.0f ? vr * vr : 0.0f;
    const float q = P.eta_damp * pp / (d * P.inv_nu_damp + P.eps);
    const float rn2 = rx * rx + ry * ry + rz * rz;
    const float mq = q * sqrtf(rn2);
    const float sigma = q / (mq + P.c * log1pf(expf(-2.0f * P.c * mq)));
    const float wl = 1.0f - d * P.inv_radius;
    const float w = d <= P.radius ? wl * wl : 0.0f;
    const float a = w * sigma * sigma;
    const float phi = P.eta_rep * expf(-d * P.inv_nu_rep) + q;
    const float bb = -a * rn2 * phi;
    csum_add(acc.s[0], acc.c[0], a * rx * rx);
    csum_add(acc.s[1], acc.c[1], a * rx * ry);
    csum_add(acc.s[2], acc.c[2], a * rx * rz);
    csum_add(acc.s[3], acc.c[3], a * ry * ry);
    csum_add(acc.s[4], acc.c[4], a * ry * rz);
    csum_add(acc.s[5], acc.c[5], a * rz * rz);
    csum_add(acc.s[6], acc.c[6], bb * rx);
    csum_add(acc.s[7], acc.c[7], bb * ry);
    csum_add(acc.s[8], acc.c[8], bb * rz);
}

// Exact "non-zero metric" predicate in float64: d < radius and xdot . r > 0, with the dot
// product evaluated left to right without fused multiply-adds.
__device__ __forceinline__ int contributes(const RayArgs &A, float rx, float ry, float rz, double d)
{
#pragma clang fp contract(off)
    const double vn = (A.vel64[0] * (double)rx + A.vel64[1] * (double)ry) + A.vel64[2] * (double)rz;
    return d < A.radius64 && vn > 0.0;
}

// Blocks are dispatched round-robin over the 8 XCDs (block b runs on XCD b % 8).  Give each
// XCD a contiguous run of tiles so that its L2 sees one compact cone of ray directions.
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

__device__ __forceinline__ FinishSlots single_slots(float *partials, uint32_t *ticket, rmpc_result *out,
                                                    uint64_t *done, uint64_t seq)
{
    FinishSlots F;
    F.tile_rows = partials;
    F.tickets = ticket;
    F.out = out;
    F.finished = nullptr;
    F.n_queries = 1;
    F.done = done;
    F.seq = seq;
    return F;
}

// A copy of *p made of wave-uniform words (readfirstlane), so that the compiler keeps it in
// scalar registers; p must be the same for every lane.
template <typename T>
__device__ __forceinline__ T load_uniform(const T *p)
{
    static_assert(sizeof(T) % 4 == 0, "whole words");
    uint32_t w[sizeof(T) / 4];
    const uint32_t *src = reinterpret_cast<const uint32_t *>(p);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w[i] = __builtin_amdgcn_readfirstlane(src[i]);
    T out;
    __builtin_memcpy(&out, w, sizeof(T));
    return out;
}

// The continuous TSDF: trilinear interpolation of the stored values, which sit at the voxel
// centres (grid coordinates i + 1/2), at grid point p; x first, then y, then z.  value(i, j, k)
// reads voxel (i, j, k) as float64 (a dense or a sparse map).
template <class Value>
__device__ __forceinline__ double trilinear_field(const Value &value, double px, double py, double pz)
{
#pragma clang fp contract(off)
    const double ux = px - 0.5, uy = py - 0.5, uz = pz - 0.5;
    const double flx = floor(ux), fly = floor(uy), flz = floor(uz);
    const int ix = (int)flx, iy = (int)fly, iz = (int)flz;
    const double fx = ux - flx, fy = uy - fly, fz = uz - flz;
    double c[2][2];
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
            const double a0 = value(ix, iy + dy, iz + dz);
            const double a1 = value(ix + 1, iy + dy, iz + dz);
            c[dz][dy] = a0 + fx * (a1 - a0);
        }
    const double e0 = c[0][0] + fy * (c[0][1] - c[0][0]);
    const double e1 = c[1][0] + fy * (c[1][1] - c[1][0]);
    return e0 + fz * (e1 - e0);
}

// Sub-voxel hit distance: the field is sampled along the ray at t_k = max(t + k/2 - 3/2, 0),
// k = 0..7 (grid units, t = d / h: from 1.5 voxels before the hit voxel's entry to 2 after
// it, a window that holds the field's zero crossing for the hits of an oblique plane); at
// the first k with phi_k > 0 >= phi_k+1 one secant step gives the crossing.  Without a sign
// change d is kept.  float64 throughout, no contraction, so the result is that of the
// definition evaluated in float64.
template <class Value>
__device__ __forceinline__ double subvoxel_at(const RayArgs &A, const Value &value, float rx, float ry, float rz,
                                              double d)
{
#pragma clang fp contract(off)
    const double t = d / A.h;
    double tk[8], phi[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const double s = t + 0.5 * (double)k - 1.5;
        tk[k] = s > 0.0 ? s : 0.0;
        phi[k] = trilinear_field(value, (double)A.g[0] + tk[k] * (double)rx, (double)A.g[1] + tk[k] * (double)ry,
                                 (double)A.g[2] + tk[k] * (double)rz);
    }
    for (int k = 0; k < 7; ++k)
        if (phi[k] > 0.0 && phi[k + 1] <= 0.0) {
            const double ts = tk[k] + (tk[k + 1] - tk[k]) * (phi[k] / (phi[k] - phi[k + 1]));
            return ts * A.h;
        }
    return d;
}

}  // namespace rmpc
