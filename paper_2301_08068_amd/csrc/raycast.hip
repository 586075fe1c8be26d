// raycast.hip -- the fused raycast-and-policy kernel (Sec. III-E, III-F), its debug twin and
// the LiDAR scan kernel (Sec. III-G).
//
// Each ray's parameter range [0, max_range / h] is split into S segments that S adjacent
// lanes walk at the same time (S = 1, 2, 4, 8 or 16): the first hit along a ray is the hit of
// the lowest segment that finds one, so a query's critical path is one segment long instead of
// one ray.  Inside a segment a lane runs a 3-D DDA (Amanatides & Woo) on the float32 start g
// and the float32 Halton direction r, in rounds that plan K steps ahead (the visited offsets
// do not depend on the loaded values, so K loads are in flight), and stops at the first
// occupied voxel, at its segment's end, at max_range or at the grid's edge.  Inside cells of
// 8 x 8 x 8 voxels and bricks of 2 x 2 x 2 voxels that the map's summaries mark free the walk
// steps cell by cell or brick by brick.  A wave
// ballot after every round stops lanes whose ray already has a hit in a lower segment.  The
// lane holding the ray's hit evaluates the obstacle policy of Sec. III-C in registers and adds
// it to compensated float32 sums; the last block to finish resolves in float64.
//
// Exactness: face crossings are compared in float32 as T = (B - g) / r with B the integer
// face coordinate (never accumulated).  When the two nearest crossings, or a crossing and
// max_range, lie within a guard band that bounds the float32 error, the decision is redone in
// float64 from the same formula, so every traversal decision -- including which axis steps at
// an exact tie (the lowest index) -- and the hit distance d = T h are the float64 values of
// the definition.  Brick and cell faces are voxel faces, so the coarse walks take the voxel
// walk's decisions restricted to them.  A segment starts at a float64-located voxel on the ray's
// walk, at a parameter chosen away from every face crossing by more than the float32 error of
// a crossing parameter, so the float32 end test of the previous segment and the start of the
// next agree exactly.

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "rmpc_device.h"
#include "rmpc_kernels.h"
#include "rmpc_sparse.h"
#include "rmpc_walk.h"

namespace rmpc {

namespace {

// The start voxel is occupied: every ray hits at distance 0 (same address for all lanes).
template <int DT>
__device__ __forceinline__ bool start_occupied(const RayArgs &A)
{
    using VT = typename Voxel<DT>::T;
    const VT *vox = static_cast<const VT *>(A.map.data);
    return Voxel<DT>::occ(vox[(uint32_t)A.lin0]);
}

// One lane's walk through one segment of one ray.  The walk moves voxel by voxel, brick by
// brick (2^3 voxels, lg = kBrickLog2) while it is inside bricks whose summary says "free", or
// cell by cell (8^3 voxels, lg = kCellLog2) inside free cells: brick and cell faces are voxel
// faces, so every level takes its decisions on the same crossing parameters and visits its
// elements in the order the voxel walk would.
struct Walker {
    int lg;                           // 0: voxel level, kBrickLog2: brick level, kCellLog2: cell level
    float Bx, By, Bz;                 // s * coordinate of the face ahead (exact integers)
    float Tx, Ty, Tz;                 // float32 parameters of those faces
    float t_exit;                     // float32 parameter of the first face on the edge of the grid
                                      // (bricks, cells: of the whole bricks, cells) that the ray crosses
    uint32_t off;                     // element offset of the current voxel, brick or cell
    int dx, dy, dz;                   // offset change of one step along each axis
    float t_hi;                       // stop once the next crossing exceeds this (float32)
    float t_lo;                       // crossings at or beyond this get the float64 range test
    bool last;                        // the segment ending at max_range
    bool pending;                     // the current voxel, brick or cell is still to be read
    int ent_a;                        // axis across which the current element was entered
    bool anchored;                    // brick or cell level: the walk is still in the element it
                                      // entered at anchor (ax, ay, az) of level anch_lg: a voxel
                                      // of the walk, or (cells only) a brick entered across anch_a
    bool settled;                     // finishing the last brick or cell voxel by voxel: no return
                                      // to coarser levels
    int ax, ay, az, anch_lg, anch_a;
    int steps;                        // decisions taken so far (orders the near-tie records)
    int tie_at, rtie_at;              // first decision index with a (range) near-tie
    // outcome
    bool ended;                       // the ray's walk ends here: a hit, max_range or the grid edge
    bool hit;
    int hit_step;                     // decision index of the step that entered the hit voxel
    int hit_a;                        // axis across which the hit voxel was entered
    int fx, fy, fz;                   // last voxel entered when ended (the hit voxel on a hit)
};

// Start walking at element (ux, uy, uz) of level lg (voxel, brick or cell).
__device__ __forceinline__ void enter_level(Walker &w, const RayF &R, const MapView &m, int lg, int ux, int uy,
                                            int uz)
{
    const float rx = R.rx, ry = R.ry, rz = R.rz;
    const int px = rx > 0.0f, py = ry > 0.0f, pz = rz > 0.0f;
    const bool cell = lg == kCellLog2, brick = lg == kBrickLog2;
    w.lg = lg;
    const int bx = (ux + px) << lg, by = (uy + py) << lg, bz = (uz + pz) << lg;
    w.Bx = (float)(px ? bx : -bx);
    w.By = (float)(py ? by : -by);
    w.Bz = (float)(pz ? bz : -bz);
    w.Tx = rx != 0.0f ? (w.Bx - R.gsx) * R.arx : kInf;
    w.Ty = ry != 0.0f ? (w.By - R.gsy) * R.ary : kInf;
    w.Tz = rz != 0.0f ? (w.Bz - R.gsz) * R.arz : kInf;
    const int vnx = m.nx, vny = m.ny, vnz = m.nz, cnx = m.ncx, cny = m.ncy, cnz = m.ncz;
    const int bnx = m.nbx, bny = m.nby, bnz = m.nbz;
    const uint32_t base = cell ? m.cell_base : (brick ? m.brick_base : 0u);
    const int nx = cell ? cnx : (brick ? bnx : vnx), ny = cell ? cny : (brick ? bny : vny);
    const int nz = cell ? cnz : (brick ? bnz : vnz);
    // the edge faces have the form of every other face, so a crossing equals t_exit exactly
    // when it is the crossing of an edge face
    const float ex = rx != 0.0f ? ((px ? (float)(nx << lg) : 0.0f) - R.gsx) * R.arx : kInf;
    const float ey = ry != 0.0f ? ((py ? (float)(ny << lg) : 0.0f) - R.gsy) * R.ary : kInf;
    const float ez = rz != 0.0f ? ((pz ? (float)(nz << lg) : 0.0f) - R.gsz) * R.arz : kInf;
    w.t_exit = fminf(ex, fminf(ey, ez));
    w.off = base + (uint32_t)ux + (uint32_t)nx * ((uint32_t)uy + (uint32_t)ny * (uint32_t)uz);
    w.dx = px ? 1 : -1;
    w.dy = py ? nx : -nx;
    w.dz = pz ? nx * ny : -(nx * ny);
}

// Integer coordinates (at the walk's level) of the position whose faces ahead are s*B.
__device__ __forceinline__ void coords_of(const RayF &R, int lg, float Bx, float By, float Bz, int &x, int &y, int &z)
{
    const int px = R.rx > 0.0f, py = R.ry > 0.0f, pz = R.rz > 0.0f;
    x = ((int)fabsf(Bx) >> lg) - px;
    y = ((int)fabsf(By) >> lg) - py;
    z = ((int)fabsf(Bz) >> lg) - pz;
}

// A round keeps which of its planned steps went along x and along y as bit masks (bit k:
// step k; the others went along z).  Undoing a set of steps is then one count per axis.
__device__ __forceinline__ int step_axis(uint32_t mx, uint32_t my, int k)
{
    return ((mx >> k) & 1u) ? 0 : (((my >> k) & 1u) ? 1 : 2);
}

// Faces ahead, and the element offset, before the steps in `sel` were taken.
__device__ __forceinline__ void undo_steps(uint32_t sel, uint32_t mx, uint32_t my, float L, int dx, int dy, int dz,
                                           float &Bx, float &By, float &Bz, uint32_t &off)
{
    const int nx = __builtin_popcount(sel & mx), ny = __builtin_popcount(sel & my);
    const int nz = __builtin_popcount(sel) - nx - ny;
    Bx -= L * (float)nx;
    By -= L * (float)ny;
    Bz -= L * (float)nz;
    off -= (uint32_t)(dx * nx + dy * ny + dz * nz);
}

// Plan K steps at the current level, load what they enter, and act on the first occupied
// voxel, brick or cell.  Returns true while the walk goes on.  The planned steps have no
// branches: the axis step is done with selects, each step's load is issued as soon as its
// offset is known, and steps past the end of the plan load a harmless offset and are ignored.
// A step whose decision needs float64 (two crossings inside the guard band, or a crossing near
// max_range) ends the plan; once the round's loads are checked, that step is taken exactly
// and what it enters is read at the start of the next round.  Only the axis of each planned
// step is kept (one bit in an x mask and a y mask); earlier positions are recovered by undoing
// later steps.
//   voxel level: an occupied voxel is the hit; a round that ends inside a free cell moves the
//     walk to the cell level, one that ends inside a free brick to the brick level.
//   brick level: an occupied brick is entered at the voxel level (its entry voxel found from
//     the crossing); a round that ends inside a free cell moves the walk to the cell level.
//   cell level: an occupied cell is entered at the brick level, in the brick that holds its
//     entry voxel.
//   brick and cell levels: at max_range or the edge of the whole bricks or cells, the current
//     free brick or cell is finished at the voxel level so that the walk's last voxel and range
//     decision are exact.
template <int DT, int K>
__device__ __forceinline__ bool walk_round(const RayArgs &A, Walker &w, const RayF &R, uint32_t safe_v,
                                           uint32_t safe_b, uint32_t safe_c)
{
    using VT = typename Voxel<DT>::T;
    const MapView &m = A.map;
    const VT *vox = static_cast<const VT *>(m.data);
    const float gx = R.gx, gy = R.gy, gz = R.gz, rx = R.rx, ry = R.ry, rz = R.rz;
    const float gsx = R.gsx, gsy = R.gsy, gsz = R.gsz, arx = R.arx, ary = R.ary, arz = R.arz;
    const int lg = w.lg;
    const bool coarse = lg != 0, cell = lg == kCellLog2;
    const float L = (float)(1 << lg);
    const uint32_t safe = cell ? safe_c : (coarse ? safe_b : safe_v);
    // the round works on copies (selects between registers, never between fields)
    float Bx = w.Bx, By = w.By, Bz = w.Bz, Tx = w.Tx, Ty = w.Ty, Tz = w.Tz;
    uint32_t off = w.off;
    const int dx = w.dx, dy = w.dy, dz = w.dz;
    const float t_exit = w.t_exit, t_hi = w.t_hi, t_lo = w.t_lo;
    // what the previous round's exact step entered is read first
    const VT pv = vox[w.pending ? off : safe];
    VT val[K];
    // The plan stops at the first step that is not simply taken: one past the segment's end,
    // near max_range (cells: the voxel level finishes there; voxels: float64 range test), on
    // an edge face, or needing float64 for a near tie.  The first three are one comparison with
    // t_stop; which of them it was is worked out again at the end of the round.
    const float t_stop = fminf(fminf(t_lo, t_exit), next_up(t_hi));
    uint32_t mx = 0, my = 0;          // planned steps along x, along y (bit k: step k)
    int nplan = 0;                    // planned steps taken
    bool going = true;                // the plan goes on
#pragma unroll
    for (int k = 0; k < K; ++k) {
        // nearest and second-nearest crossings (no NaNs occur: +inf marks an axis never crossed)
        const float t1 = __builtin_amdgcn_fmed3f(Tx, fminf(Ty, Tz), -kInf);
        const float t2 = __builtin_amdgcn_fmed3f(Tx, Ty, Tz);
        // (bitwise operators: no short-circuit branches in the plan)
        const bool bx = Tx == t1, by = !bx & (Ty == t1), bz = !bx & !by;
        going = going & (t1 < t_stop) & (t2 - t1 >= 2e-5f + 1e-6f * t2);
        Bx = bx ? Bx + L : Bx;
        By = by ? By + L : By;
        Bz = bz ? Bz + L : Bz;
        Tx = bx ? (Bx - gsx) * arx : Tx;
        Ty = by ? (By - gsy) * ary : Ty;
        Tz = bz ? (Bz - gsz) * arz : Tz;
        off += (uint32_t)(bx ? dx : (by ? dy : dz));
        val[k] = vox[going ? off : safe];
        mx |= bx ? 1u << k : 0u;
        my |= by ? 1u << k : 0u;
        nplan += going ? 1 : 0;
        in_vgpr(mx);
        in_vgpr(my);
        in_vgpr(nplan);
    }
    // after a full round: the summaries of the cell (voxel and brick levels) and of the brick
    // (voxel level) the walk is in, for a move to a coarser level, loaded before the plan's
    // values are examined
    int ux, uy, uz;                   // the walk's element at its level
    coords_of(R, lg, Bx, By, Bz, ux, uy, uz);
    const int csh = kCellLog2 - lg;
    const int ccx = ux >> csh, ccy = uy >> csh, ccz = uz >> csh;
    const bool cin = !cell && going && ccx < m.ncx && ccy < m.ncy && ccz < m.ncz;
    const VT cf = vox[cin ? m.cell_base + (uint32_t)ccx + (uint32_t)m.ncx * ((uint32_t)ccy + (uint32_t)m.ncy * (uint32_t)ccz)
                          : safe_c];
    const int bcx = ux >> kBrickLog2, bcy = uy >> kBrickLog2, bcz = uz >> kBrickLog2;
    const bool bin = !coarse && going && bcx < m.nbx && bcy < m.nby && bcz < m.nbz;
    const VT bf = vox[bin ? m.brick_base + (uint32_t)bcx + (uint32_t)m.nbx * ((uint32_t)bcy + (uint32_t)m.nby * (uint32_t)bcz)
                          : safe_b];
    uint32_t occm = 0;                // planned steps that entered an occupied element
#pragma unroll
    for (int k = 0; k < K; ++k) occm |= Voxel<DT>::occ(val[k]) ? 1u << k : 0u;
    occm &= (1u << nplan) - 1u;
    const int hk = occm ? __builtin_ctz(occm) : -1;
    const int steps = w.steps;

    // Each case below only records what happens; the shared tail then computes an entry voxel
    // and moves the walk to its new level once, whatever mix of cases a wave's lanes take.
    bool go_on = false;               // the walk continues next round
    bool hit_now = false;             // the hit voxel (hx, hy, hz), entered across axis ha
    int hx = 0, hy = 0, hz = 0, ha = 0;
    int to_level = -1;                // >= 0: continue at this level, in the element that holds
    int tx = 0, ty = 0, tz = 0;       //   voxel (tx, ty, tz)
    int entry_lg = 0;                 // > 0: that voxel is the entry voxel of element (ex, ey, ez)
    int ex = 0, ey = 0, ez = 0;       //   of this level, entered across axis ta_
    int ta_ = 0;
    int entry_tie_at = -1;            // decision index of that entry, for its near-tie record (-1: none)
    bool to_pending = false;          // the element the walk continues in is still to be read
    int anch = -1;                    // >= 0: level of the new anchor (nax, nay, naz), axis naa
    int nax = 0, nay = 0, naz = 0, naa = 0;

    const bool pending_hit = w.pending && Voxel<DT>::occ(pv);
    w.pending = false;
    // Every case continues from the position after one step j of the plan: the step that
    // entered the first occupied element, the last step taken, or none (j = -1: the round's
    // start, which is the element the previous round's exact step entered).  The plan applied
    // all K steps to (B, off), so the later ones are undone once here for all lanes.
    const int j = pending_hit ? -1 : (hk >= 0 ? hk : nplan - 1);
    undo_steps(((1u << K) - 1u) & ~(j >= 0 ? (2u << j) - 1u : 0u), mx, my, L, dx, dy, dz, Bx, By, Bz, off);
    int jx, jy, jz;                   // the element after step j, entered across axis aj
    coords_of(R, lg, Bx, By, Bz, jx, jy, jz);
    const int aj = j >= 0 ? step_axis(mx, my, j) : w.ent_a;
    if (pending_hit || hk >= 0) {
        // (a, b) the element entered at decision steps + j is occupied: the voxel, brick or cell
        // entered by the previous round's exact step (or, for a brick, by the descent from its
        // cell), or the first occupied one among the planned steps
        w.steps = steps + j + 1;
        go_on = coarse;
        if (!coarse) {
            hit_now = true;
            hx = jx; hy = jy; hz = jz; ha = aj;
            w.hit_step = steps + j;
        } else if (pending_hit && !cell && w.anchored) {
            // a brick entered from its cell: the cell's entry voxel is the brick's
            to_level = 0; to_pending = true;
            tx = w.ax; ty = w.ay; tz = w.az; ta_ = aj;
        } else {
            to_level = cell ? kBrickLog2 : 0; to_pending = true;
            entry_lg = lg; ex = jx; ey = jy; ez = jz; ta_ = aj;
            entry_tie_at = steps + j;
        }
    } else if (nplan == K) {
        // (c) a full round: continue, at a coarser level if the walk is inside a free cell or
        // (voxel level) a free brick
        w.Bx = Bx; w.By = By; w.Bz = Bz; w.Tx = Tx; w.Ty = Ty; w.Tz = Tz;
        w.off = off;
        w.steps = steps + K;
        go_on = true;
        if (coarse) {
            w.anchored = false;
            w.ent_a = aj;
        }
        if (!cell && !w.settled && cin && !Voxel<DT>::occ(cf)) {
            to_level = kCellLog2;
            tx = ux << lg; ty = uy << lg; tz = uz << lg;
            anch = lg; nax = ux; nay = uy; naz = uz; naa = aj;
        } else if (!coarse && !w.settled && bin && !Voxel<DT>::occ(bf)) {
            to_level = kBrickLog2;
            tx = ux; ty = uy; tz = uz;
            anch = 0; nax = ux; nay = uy; naz = uz;
        }
    } else {
        // (d) the plan ended at step nplan: continue from the position after step nplan - 1
        Tx = rx != 0.0f ? (Bx - gsx) * arx : kInf;
        Ty = ry != 0.0f ? (By - gsy) * ary : kInf;
        Tz = rz != 0.0f ? (Bz - gsz) * arz : kInf;
        // why the plan stopped at step nplan, from the same crossings the plan saw there
        const float t1 = __builtin_amdgcn_fmed3f(Tx, fminf(Ty, Tz), -kInf);
        const float t2 = __builtin_amdgcn_fmed3f(Tx, Ty, Tz);
        const bool near_end = t1 >= t_lo;
        const bool stop_n = (t1 > t_hi) | (coarse & near_end);
        const bool need64 = (t2 - t1 < 2e-5f + 1e-6f * t2) | (!coarse & near_end);
        const bool hard = !stop_n & need64;
        // past the float64 cases an edge-face crossing is not tied, so t1 names it exactly
        bool exited = !stop_n & !need64 & (t1 >= t_exit);
        int tie_at = w.tie_at, rtie_at = w.rtie_at;
        bool taken = false;
        if (hard) {
            // the step the plan stopped at, decided in float64 exactly as the definition does
            const int at = steps + nplan;
            int a = Tx == t1 ? 0 : (Ty == t1 ? 1 : 2);
            bool tie = false;
            if (t2 - t1 < 2e-5f + 1e-6f * t2) {
                const double X = rx != 0.0f ? face64((int)fabsf(Bx), gx, rx) : __builtin_huge_val();
                const double Y = ry != 0.0f ? face64((int)fabsf(By), gy, ry) : __builtin_huge_val();
                const double Z = rz != 0.0f ? face64((int)fabsf(Bz), gz, rz) : __builtin_huge_val();
                a = 0;
                double m1 = X;
                if (Y < m1) { a = 1; m1 = Y; }
                if (Z < m1) { a = 2; m1 = Z; }
                tie = (a != 0 && X - m1 < 1e-5) || (a != 1 && Y - m1 < 1e-5) || (a != 2 && Z - m1 < 1e-5);
            }
            // near-ties count at every voxel decision, at the brick and cell levels only on
            // steps taken
            if (tie && !coarse) tie_at = min(tie_at, at);
            const float ta = a == 0 ? Tx : (a == 1 ? Ty : Tz);
            bool stop = ta > t_hi || (coarse && ta >= t_lo);
            if (!coarse && !stop && ta >= t_lo) {
                // range test (closed interval) in float64 inside the guard band
                const double T64 = a == 0 ? face64((int)fabsf(Bx), gx, rx)
                                          : (a == 1 ? face64((int)fabsf(By), gy, ry) : face64((int)fabsf(Bz), gz, rz));
                const double dist = T64 * A.h;
                stop = dist > A.max_range;
                if (fabs(dist - A.max_range) < 1e-5 * A.h) rtie_at = min(rtie_at, at);
            }
            if (!stop) {
                const float nBx = a == 0 ? Bx + L : Bx, nBy = a == 1 ? By + L : By, nBz = a == 2 ? Bz + L : Bz;
                // the face crossed is an edge face when the new face ahead lies past the edge
                // (the sizes pass through readfirstlane as values: a select among fields of the
                // kernel argument would become an indexed load from a private copy of it)
                const int vnx = __builtin_amdgcn_readfirstlane(m.nx), vny = __builtin_amdgcn_readfirstlane(m.ny);
                const int vnz = __builtin_amdgcn_readfirstlane(m.nz), cnx = __builtin_amdgcn_readfirstlane(m.ncx);
                const int cny = __builtin_amdgcn_readfirstlane(m.ncy), cnz = __builtin_amdgcn_readfirstlane(m.ncz);
                const int bnx = __builtin_amdgcn_readfirstlane(m.nbx), bny = __builtin_amdgcn_readfirstlane(m.nby);
                const int bnz = __builtin_amdgcn_readfirstlane(m.nbz);
                const int pa = a == 0 ? rx > 0.0f : (a == 1 ? ry > 0.0f : rz > 0.0f);
                const int nxl = cell ? cnx : (coarse ? bnx : vnx), nyl = cell ? cny : (coarse ? bny : vny);
                const int nzl = cell ? cnz : (coarse ? bnz : vnz);
                const int na = a == 0 ? nxl : (a == 1 ? nyl : nzl);
                const float edge = pa ? (float)(na << lg) : 0.0f;
                if ((a == 0 ? nBx : (a == 1 ? nBy : nBz)) <= edge) {
                    // take it; the next round reads what it enters
                    if (tie && coarse) tie_at = min(tie_at, at);
                    w.Bx = nBx; w.By = nBy; w.Bz = nBz;
                    w.Tx = a == 0 && rx != 0.0f ? (nBx - gsx) * arx : Tx;
                    w.Ty = a == 1 && ry != 0.0f ? (nBy - gsy) * ary : Ty;
                    w.Tz = a == 2 && rz != 0.0f ? (nBz - gsz) * arz : Tz;
                    w.off = off + (uint32_t)(a == 0 ? dx : (a == 1 ? dy : dz));
                    w.pending = true;
                    w.ent_a = a;
                    w.anchored = false;
                    w.steps = at + 1;
                    taken = true;
                    go_on = true;
                } else {
                    exited = true;
                }
            }
        }
        w.tie_at = tie_at;
        w.rtie_at = rtie_at;
        if (!taken) {
            // (e) the walk stops in this segment after step nplan - 1 (max_range, segment end,
            // or the edge of the grid or of the whole bricks or cells)
            w.steps = steps + nplan;
            if (!coarse) {
                if (w.last || exited) {
                    coords_of(R, 0, Bx, By, Bz, w.fx, w.fy, w.fz);        // the last voxel entered
                    w.ended = true;
                }
            } else if (w.last || exited) {
                // finish the current (free) brick or cell voxel by voxel: the walk ends in it or
                // just past it (max range, or the grid edge beyond the whole bricks or cells),
                // so it stays at the voxel level
                w.settled = true;
                to_level = 0;
                go_on = true;
                if (nplan == 0 && w.anchored) {
                    if (w.anch_lg == 0) {
                        tx = w.ax; ty = w.ay; tz = w.az;
                    } else {
                        entry_lg = w.anch_lg; ex = w.ax; ey = w.ay; ez = w.az; ta_ = w.anch_a;
                    }
                } else {
                    entry_lg = lg;
                    ex = jx; ey = jy; ez = jz; ta_ = aj;
                }
            }
        }
    }
    if (hit_now) {
        w.fx = hx; w.fy = hy; w.fz = hz;
        w.hit_a = ha;
        w.hit = w.ended = true;
        return false;
    }
    if (entry_lg != 0) {
        bool tie = false;
        int vx, vy, vz;
        entry_voxel(A, R, entry_lg, ta_, ex, ey, ez, vx, vy, vz, tie);
        if (tie && entry_tie_at >= 0) w.tie_at = min(w.tie_at, entry_tie_at);
        tx = vx; ty = vy; tz = vz;
        if (to_level == kBrickLog2) { anch = 0; nax = vx; nay = vy; naz = vz; }    // a cell's entry voxel
    }
    if (to_level >= 0) {
        enter_level(w, R, m, to_level, tx >> to_level, ty >> to_level, tz >> to_level);
        w.anchored = anch >= 0;
        w.anch_lg = anch; w.anch_a = naa;
        w.ax = nax; w.ay = nay; w.az = naz;
        w.pending = to_pending;
        w.ent_a = ta_;
    }
    return go_on;
}

// Per-ray outcome, valid in the lane that reports the ray (its hit segment, else segment 0).
struct RayOut {
    bool report;
    bool hit;
    double d;
    uint32_t flags;
    int visits_lane;                  // the ray's visit count in one lane of its group, else 0
    int hit_lin;                      // debug
};

// Walk one ray with the S lanes of its group; every lane of the wave must call this.
template <int DT, int K>
__device__ __forceinline__ RayOut trace_group(const RayArgs &A, bool valid, int seg, int S,
                                              float rx, float ry, float rz)
{
    using VT = typename Voxel<DT>::T;
    const MapView &m = A.map;
    const RayF R = make_ray(A, rx, ry, rz);
    const double tmax = A.tmax_v;
    Walker w;
    w.pending = false;
    w.ent_a = 0;
    w.anchored = false;
    w.settled = false;
    w.ax = w.ay = w.az = 0;
    w.anch_lg = w.anch_a = 0;
    w.steps = 0;
    w.tie_at = w.rtie_at = 1 << 30;
    w.ended = false;
    w.hit = false;
    w.hit_step = -1;
    w.hit_a = 0;
    w.fx = w.fy = w.fz = 0;
    bool active = valid;
    const VT *vox = static_cast<const VT *>(m.data);
    const uint32_t safe_v = A.lin0;
    const uint32_t safe_c = m.ncx > 0 && m.ncy > 0 && m.ncz > 0 ? m.cell_base : safe_v;
    const uint32_t safe_b = m.nbx > 0 && m.nby > 0 && m.nbz > 0 ? m.brick_base : safe_v;
    // the summaries of the start voxel's cell and brick: the same for every segment-0 lane
    // (issued now, while the segment bounds are computed)
    const int c0x = A.v0[0] >> kCellLog2, c0y = A.v0[1] >> kCellLog2, c0z = A.v0[2] >> kCellLog2;
    const bool c0in = c0x < m.ncx && c0y < m.ncy && c0z < m.ncz;
    const VT cf0 = vox[c0in ? m.cell_base + (uint32_t)c0x + (uint32_t)m.ncx * ((uint32_t)c0y + (uint32_t)m.ncy * (uint32_t)c0z)
                            : safe_c];
    const int b0x = A.v0[0] >> kBrickLog2, b0y = A.v0[1] >> kBrickLog2, b0z = A.v0[2] >> kBrickLog2;
    const bool b0in = b0x < m.nbx && b0y < m.nby && b0z < m.nbz;
    const VT bf0 = vox[b0in ? m.brick_base + (uint32_t)b0x + (uint32_t)m.nbx * ((uint32_t)b0y + (uint32_t)m.nby * (uint32_t)b0z)
                            : safe_b];
    // segment start
    int ux = A.v0[0], uy = A.v0[1], uz = A.v0[2];
    if (seg != 0) {
        bool ok;
        seg_boundary(tmax * seg / S, R.gx, R.gy, R.gz, rx, ry, rz, ux, uy, uz, ok);
        if (!ok || (unsigned)ux >= (unsigned)m.nx || (unsigned)uy >= (unsigned)m.ny || (unsigned)uz >= (unsigned)m.nz) {
            active = false;                               // empty segment (or past the grid)
            ux = A.v0[0]; uy = A.v0[1]; uz = A.v0[2];
        }
    }
    // segment end: the next boundary that exists, else max_range
    w.last = true;
    w.t_hi = A.tmax_hi;
    w.t_lo = A.tmax_lo;
    for (int e = seg + 1; e < S && w.last; ++e) {
        int bx, by, bz;
        bool ok;
        const double te = seg_boundary(tmax * e / S, R.gx, R.gy, R.gz, rx, ry, rz, bx, by, bz, ok);
        if (ok) {
            w.last = false;
            w.t_hi = (float)te;       // no crossing lies within the segment margin of te
            w.t_lo = kInf;
        }
    }
    // every segment starts at the coarsest level whose element around its start voxel is free
    // (a later segment reads those summaries once its start voxel is known), anchored at the
    // start voxel
    int scx = c0x, scy = c0y, scz = c0z, sbx = b0x, sby = b0y, sbz = b0z;
    bool sc_in = c0in, sb_in = b0in;
    VT cf = cf0, bf = bf0;
    if (seg != 0) {
        scx = ux >> kCellLog2; scy = uy >> kCellLog2; scz = uz >> kCellLog2;
        sbx = ux >> kBrickLog2; sby = uy >> kBrickLog2; sbz = uz >> kBrickLog2;
        sc_in = scx < m.ncx && scy < m.ncy && scz < m.ncz;
        sb_in = sbx < m.nbx && sby < m.nby && sbz < m.nbz;
        cf = vox[sc_in ? m.cell_base + (uint32_t)scx + (uint32_t)m.ncx * ((uint32_t)scy + (uint32_t)m.ncy * (uint32_t)scz)
                       : safe_c];
        bf = vox[sb_in ? m.brick_base + (uint32_t)sbx + (uint32_t)m.nbx * ((uint32_t)sby + (uint32_t)m.nby * (uint32_t)sbz)
                       : safe_b];
    }
    const bool start_cell = sc_in && !Voxel<DT>::occ(cf), start_brick = !start_cell && sb_in && !Voxel<DT>::occ(bf);
    if (start_cell) enter_level(w, R, m, kCellLog2, scx, scy, scz);
    else if (start_brick) enter_level(w, R, m, kBrickLog2, sbx, sby, sbz);
    else enter_level(w, R, m, 0, ux, uy, uz);
    w.anchored = start_cell || start_brick;
    w.ax = ux; w.ay = uy; w.az = uz;

    const int lane = threadIdx.x & (kWave - 1);
    const int base = lane & ~(S - 1);
    const uint64_t seg_bits = (1ull << S) - 1ull;        // S <= 16
    const uint64_t lower = ((1ull << seg) - 1ull) << base;
    for (;;) {
        const uint64_t hm = __ballot(w.hit);
        if (hm & lower) active = false;                  // a lower segment already hit
        if (!__any(active)) break;
        if (active) active = walk_round<DT, K>(A, w, R, safe_v, safe_b, safe_c);
    }
    // combine the group: the lowest segment with a hit owns the ray; the lowest segment whose
    // walk ended holds the ray's last voxel
    const uint64_t gh = (__ballot(w.hit) >> base) & seg_bits;
    const int h = gh ? __ffsll((unsigned long long)gh) - 1 : S;
    const uint64_t ge = (__ballot(valid && w.ended) >> base) & seg_bits;
    const int t = ge ? __ffsll((unsigned long long)ge) - 1 : S;
    const bool keep = valid && seg <= h;
    RayOut o;
    // voxels entered, start voxel included: every step changes one coordinate by one toward
    // the ray's direction, so the count follows from the first and the last voxel
    o.visits_lane = valid && seg == t ? 1 + abs(w.fx - A.v0[0]) + abs(w.fy - A.v0[1]) + abs(w.fz - A.v0[2]) : 0;
    const bool tie = keep && w.tie_at <= (seg == h ? w.hit_step : (1 << 29));
    const bool rtie = keep && w.rtie_at <= (seg == h ? w.hit_step : (1 << 29));
    const uint64_t tm = (__ballot(tie) >> base) & seg_bits;
    const uint64_t rm = (__ballot(rtie) >> base) & seg_bits;
    o.report = valid && seg == (h < S ? h : 0);
    o.hit = w.hit && seg == h;
    // the hit distance: the float64 parameter of the face through which the hit voxel was
    // entered, in metres
    double d = __builtin_huge_val();
    if (o.hit) {
        const double T64 = w.hit_a == 0 ? entry64(w.fx, R.gx, R.rx)
                                        : (w.hit_a == 1 ? entry64(w.fy, R.gy, R.ry) : entry64(w.fz, R.gz, R.rz));
        d = T64 * A.h;
    }
    o.d = d;
    o.flags = A.start_flags | (tm ? kRayTie : 0u) | (rm ? kRayRangeTie : 0u);
    o.hit_lin = o.hit ? w.fx + m.nx * (w.fy + m.ny * w.fz) : -1;
    return o;
}

// The stored value of voxel (i, j, k) of a dense map, the indices clamped into the grid, as
// float64 (exact for float32 and binary16): the field reader of sub-voxel distances.
template <int DT>
struct DenseField {
    const typename Voxel<DT>::T *data;
    int nx, ny, nz;
    __device__ __forceinline__ double operator()(int i, int j, int k) const
    {
        i = i < 0 ? 0 : (i >= nx ? nx - 1 : i);
        j = j < 0 ? 0 : (j >= ny ? ny - 1 : j);
        k = k < 0 ? 0 : (k >= nz ? nz - 1 : k);
        const typename Voxel<DT>::T v = data[(uint32_t)i + (uint32_t)nx * ((uint32_t)j + (uint32_t)ny * (uint32_t)k)];
        if constexpr (DT == RMPC_TSDF_F32) return (double)v;
        else return (double)__builtin_bit_cast(_Float16, v);
    }
};

template <int DT>
__device__ __forceinline__ double subvoxel_distance(const RayArgs &A, float rx, float ry, float rz, double d)
{
    const DenseField<DT> f{static_cast<const typename Voxel<DT>::T *>(A.map.data), A.map.nx, A.map.ny, A.map.nz};
    return subvoxel_at(A, f, rx, ry, rz, d);
}

// One 256-lane tile of a map query: lane -> (ray position, segment).  Waves stay whole (the
// traversal uses wave-wide ballots); lanes past the end, or whose list entry is >= n_rays,
// take part as idle members.  A lane traces first and only then holds accumulators.
template <int DT, int K>
__device__ __forceinline__ void ray_tile(const RayArgs &A, int tile, int n_tiles, const FinishSlots &F,
                                         float *lds)
{
    const bool in_coll = start_occupied<DT>(A);
    const int S = A.segments;
    const int p = tile * kBlock + threadIdx.x;
    const int j = p < A.n_list * S ? p / S : 0;
    const int seg = p & (S - 1);
    const float4 rr = load_ray(A.rays, j);
    const bool valid = p < A.n_list * S && __float_as_int(rr.w) < A.n_rays;
    const float rx = rr.x, ry = rr.y, rz = rr.z;
    Acc acc;
    acc.zero();
    if (in_coll) {
        if (valid && seg == 0) {
            acc.visits = 1;
            acc.n_hit = 1;
            acc.n_contrib = contributes(A, rx, ry, rz, 0.0);
            policy_accumulate(A.pol, rx, ry, rz, 0.0f, acc);
        }
    } else {
        const RayOut o = trace_group<DT, K>(A, valid, seg, S, rx, ry, rz);
        acc.visits = o.visits_lane;
        if (o.report) {
            acc.n_tie = (o.flags & kRayTie) != 0;
            if (o.hit) {
                double d = o.d;
                if constexpr (DT != RMPC_OCC_U8)
                    if (A.subvoxel) d = subvoxel_distance<DT>(A, rx, ry, rz, d);
                acc.n_hit = 1;
                acc.n_contrib = contributes(A, rx, ry, rz, d);
                policy_accumulate(A.pol, rx, ry, rz, (float)d, acc);
            }
        }
    }
    grid_finish(acc, tile, n_tiles, F, A.rank_tol, A.n_rays, in_coll ? RMPC_Q_IN_COLLISION : 0u, lds);
}

// One tile of a LiDAR scan query (Sec. III-G): point p gives direction p/|p| and distance
// |p|; non-finite points and points closer than min_range are skipped.  Tile t covers points
// t*256 + lane + k * n_tiles * 256, which a thread takes in increasing k.  A thread loads
// kScanBatch of its points before it evaluates the first, so that their loads wait once.
__device__ __forceinline__ void scan_tile(const ScanArgs &A, int tile, int n_tiles, const FinishSlots &F,
                                          float *lds)
{
    Acc acc;
    acc.zero();
    const int stride = n_tiles * kBlock;
    for (int i0 = tile * kBlock + threadIdx.x; i0 < A.n_points; i0 += kScanBatch * stride) {
        float p[kScanBatch][3];
#pragma unroll
        for (int k = 0; k < kScanBatch; ++k) {
            const int i = i0 + k * stride;
            const size_t j = i < A.n_points ? 3 * (size_t)i : 0;      // past the end: point 0, unused
            p[k][0] = A.points[j];
            p[k][1] = A.points[j + 1];
            p[k][2] = A.points[j + 2];
        }
#pragma unroll
        for (int k = 0; k < kScanBatch; ++k) {
            const float px = p[k][0], py = p[k][1], pz = p[k][2];
            if (i0 + k * stride >= A.n_points || !(isfinite(px) && isfinite(py) && isfinite(pz))) continue;
            double n2, vp;
            {
#pragma clang fp contract(off)
                n2 = ((double)px * (double)px + (double)py * (double)py) + (double)pz * (double)pz;
                vp = (A.vel64[0] * (double)px + A.vel64[1] * (double)py) + A.vel64[2] * (double)pz;
            }
            if (!(n2 >= A.min_range2)) continue;
            const double d64 = sqrt(n2);
            const float inv = (float)(1.0 / d64);
            acc.n_hit += 1;
            acc.n_contrib += d64 < A.radius64 && vp > 0.0;
            policy_accumulate(A.pol, px * inv, py * inv, pz * inv, (float)d64, acc);
        }
    }
    grid_finish(acc, tile, n_tiles, F, A.rank_tol, A.n_points, 0u, lds);
}

// One map query per launch; block b takes tile xcd_tile(b).
template <int DT, int K>
// One 65,536-ray query at the default lane target has 2 waves per SIMD, so the kernel is built
// for 2: the register budget then fits lookahead 16 without spills (lookahead 4 and 8 still
// stay within 128 registers, 4 waves per SIMD).
__global__ void __launch_bounds__(kBlock, 2) raycast_rmp_kernel(RayArgs A)
{
    __shared__ float lds[kReduceLdsWords];
    ray_tile<DT, K>(A, xcd_tile(blockIdx.x, gridDim.x), gridDim.x,
                    single_slots(A.partials, A.ticket, A.result, A.done, A.seq), lds);
}

// Many map and scan queries in one persistent launch: resident blocks take tiles from a
// counter (work[0]) until none are left; tile rows, tickets and results are per query, so a
// query's result does not depend on which block ran which tile.  The last block to leave
// resets the counters for the next launch.
template <int K>
__global__ void __launch_bounds__(kBlock, 3) batch_kernel(BatchArgs B)
{
    __shared__ float lds[kReduceLdsWords];
    __shared__ int s_tile;
    const int n_tiles = B.hdr->n_tiles;
    const int n_queries = B.hdr->n_queries;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0)
            s_tile = (int)__hip_atomic_fetch_add(B.work, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        // the tile and its query are the same for the whole block: keep them (and the query's
        // descriptor loads) in scalar registers
        const int tile = __builtin_amdgcn_readfirstlane(s_tile);
        if (tile >= n_tiles) break;
        int lo = 0, hi = n_queries - 1;      // last query with tile_begin <= tile
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (B.q[mid].tile_begin <= tile) lo = mid; else hi = mid - 1;
        }
        lo = __builtin_amdgcn_readfirstlane(lo);
        const BatchQuery &Qm = B.q[lo];
        const int q_tile_begin = Qm.tile_begin, q_n_tiles = Qm.n_tiles, q_kind = Qm.kind;
        FinishSlots F;
        F.tile_rows = B.partials + (size_t)q_tile_begin * kPartialWords;
        F.tickets = B.tickets + lo;
        F.out = B.results + lo;
        F.finished = B.work + 2;
        F.n_queries = n_queries;
        F.done = B.done;
        F.seq = B.hdr->seq;
        const int t = tile - q_tile_begin;
        // the descriptor is the same for the whole block: copy it into scalar registers
        if (q_kind == 0) {
            const RayArgs A = load_uniform(&Qm.ray);
            if (A.sparse) {
                // block rounds of 4 steps on sparse maps (their best; larger ones would raise the
                // kernel's register budget and make the dense path spill), no sub-voxel
                // refinement (batches refuse it on sparse maps, for the same reason)
                sparse_tile<4, kSvNone>(A, t, q_n_tiles, F, lds);
                continue;
            }
            switch (A.map.dtype) {
            case RMPC_TSDF_F32: ray_tile<RMPC_TSDF_F32, K>(A, t, q_n_tiles, F, lds); break;
            case RMPC_TSDF_F16: ray_tile<RMPC_TSDF_F16, K>(A, t, q_n_tiles, F, lds); break;
            default: ray_tile<RMPC_OCC_U8, K>(A, t, q_n_tiles, F, lds); break;
            }
        } else {
            const ScanArgs A = load_uniform(&Qm.scan);
            scan_tile(A, t, q_n_tiles, F, lds);
        }
    }
    if (threadIdx.x == 0) {
        const uint32_t prev = __hip_atomic_fetch_add(B.work + 1, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == gridDim.x - 1) {
            __hip_atomic_store(B.work, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(B.work + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <int DT, int K>
__global__ void __launch_bounds__(kBlock, 2) trace_debug_kernel(RayArgs A)
{
    const int S = A.segments;
    const int p = xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    const int j = p < A.n_list * S ? p / S : 0;
    const int seg = p & (S - 1);
    const float4 rr = load_ray(A.rays, j);
    const int i = __float_as_int(rr.w);
    const bool valid = p < A.n_list * S && i < A.n_rays;
    const float rx = rr.x, ry = rr.y, rz = rr.z;
    if (start_occupied<DT>(A)) {
        if (valid && seg == 0) {
            A.dbg_hit[i] = A.lin0;
            A.dbg_dist[i] = 0.0;
            A.dbg_flags[i] = (uint8_t)(A.start_flags | kRayInCollision);
            if (A.dbg_visits) A.dbg_visits[i] = 1;
        }
        return;
    }
    const RayOut o = trace_group<DT, K>(A, valid, seg, S, rx, ry, rz);
    // the ray's visit count is the sum over its group
    int v = o.visits_lane;
    for (int off = 1; off < S; off <<= 1) v += __shfl_xor(v, off, kWave);
    if (o.report) {
        A.dbg_hit[i] = o.hit ? o.hit_lin : -1;
        double d = o.d;
        if constexpr (DT != RMPC_OCC_U8)
            if (A.subvoxel && o.hit) d = subvoxel_distance<DT>(A, rx, ry, rz, d);
        A.dbg_dist[i] = d;
        A.dbg_flags[i] = (uint8_t)o.flags;
        if (A.dbg_visits) A.dbg_visits[i] = v;
    }
}

// One scan query per launch.
__global__ void __launch_bounds__(kBlock) scan_rmp_kernel(ScanArgs A)
{
    __shared__ float lds[kReduceLdsWords];
    scan_tile(A, blockIdx.x, gridDim.x, single_slots(A.partials, A.ticket, A.result, A.done, A.seq), lds);
}

template <int DT, int K>
hipError_t launch_k(const RayArgs &A, int grid, hipStream_t s, bool debug, hipEvent_t e0, hipEvent_t e1)
{
    const dim3 blk(kBlock);
    if (debug) {
        const dim3 g((A.n_list * A.segments + kBlock - 1) / kBlock);
        if (e0) hipExtLaunchKernelGGL(trace_debug_kernel<DT, K>, g, blk, 0, s, e0, e1, 0, A);
        else trace_debug_kernel<DT, K><<<g, blk, 0, s>>>(A);
    } else {
        if (e0) hipExtLaunchKernelGGL(raycast_rmp_kernel<DT, K>, dim3(grid), blk, 0, s, e0, e1, 0, A);
        else raycast_rmp_kernel<DT, K><<<grid, blk, 0, s>>>(A);
    }
    return hipGetLastError();
}

template <int DT>
hipError_t launch_dt(const RayArgs &A, int grid, hipStream_t s, bool debug, hipEvent_t e0, hipEvent_t e1)
{
    switch (A.lookahead) {
    case 4: return launch_k<DT, 4>(A, grid, s, debug, e0, e1);
    case 16: return launch_k<DT, 16>(A, grid, s, debug, e0, e1);
    default: return launch_k<DT, 8>(A, grid, s, debug, e0, e1);
    }
}

}  // namespace

int ray_grid_blocks(int lanes)
{
    int b = (lanes + kBlock - 1) / kBlock;
    return b < 1 ? 1 : (b > kMaxBlocks ? kMaxBlocks : b);
}

// At most 128 blocks: every block pays a ticket with an agent-scope release and acquire at the
// end, which costs more than looping over a few more points per thread (measured: 262,144
// points take 19.5 us with 128 blocks against 43 us with 1024; 65,536 points 13.6 against 17.6).
int scan_grid_blocks(int n_points)
{
    int b = (n_points + kBlock - 1) / kBlock;
    return b < 1 ? 1 : (b > kScanMaxBlocks ? kScanMaxBlocks : b);
}

hipError_t launch_scan(const ScanArgs &A, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    const dim3 g(scan_grid_blocks(A.n_points)), blk(kBlock);
    if (e0) hipExtLaunchKernelGGL(scan_rmp_kernel, g, blk, 0, s, e0, e1, 0, A);
    else scan_rmp_kernel<<<g, blk, 0, s>>>(A);
    return hipGetLastError();
}

int batch_blocks_per_cu(int lookahead)
{
    int nb = 0;
    hipError_t e;
    switch (lookahead) {
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_kernel<4>, kBlock, 0); break;
    case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_kernel<16>, kBlock, 0); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_kernel<8>, kBlock, 0); break;
    }
    return e == hipSuccess && nb > 0 ? nb : 1;
}

hipError_t launch_batch(const BatchArgs &a, int blocks, int lookahead, hipStream_t s)
{
    switch (lookahead) {
    case 4: batch_kernel<4><<<blocks, kBlock, 0, s>>>(a); break;
    case 16: batch_kernel<16><<<blocks, kBlock, 0, s>>>(a); break;
    default: batch_kernel<8><<<blocks, kBlock, 0, s>>>(a); break;
    }
    return hipGetLastError();
}

hipError_t launch_raycast(const RayArgs &A, hipStream_t s, bool debug, hipEvent_t e0, hipEvent_t e1)
{
    const int grid = ray_grid_blocks(A.n_list * A.segments);
    switch (A.map.dtype) {
    case RMPC_TSDF_F32: return launch_dt<RMPC_TSDF_F32>(A, grid, s, debug, e0, e1);
    case RMPC_TSDF_F16: return launch_dt<RMPC_TSDF_F16>(A, grid, s, debug, e0, e1);
    default: return launch_dt<RMPC_OCC_U8>(A, grid, s, debug, e0, e1);
    }
}

}  // namespace rmpc
