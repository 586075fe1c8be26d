// rollout.hip -- closed-loop rollout (Sec. III-A Eq. 1 with the goal attractor of Sec. III-C
// Eqs. 3-4): every state's ray policy comes from a query launch; the attractor, the 3x3 solve
// and the integration are a few float64 operations on the host around it.  A single flight
// runs one rmpc_query per step; a batch of flights runs one rmpc_query_batch per step over the
// flights still flying.  Both drive the same per-flight state machine, so their outcomes agree
// whenever the query results do.

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "rmpc_host.h"

using rmpc_host::fail;
using rmpc_host::finite3;

namespace {

constexpr double kPi = 3.14159265358979323846;

// Eq. 4: s(u) = u / (|u| + c log(1 + exp(-2 c |u|))).
void soft_normalize(const double u[3], double c, double out[3])
{
    const double m = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const double den = m + c * std::log1p(std::exp(-2.0 * c * m));
    for (int i = 0; i < 3; ++i) out[i] = den > 0.0 ? u[i] / den : 0.0;
}

// y = (I + A)^-1 r for a symmetric positive semi-definite A (row major), by Cholesky of the
// positive definite I + A.  False when the factorisation breaks down (A not PSD or not finite).
bool solve_identity_plus(const double A[9], const double r[3], double y[3])
{
    double L[3][3] = {};
    for (int j = 0; j < 3; ++j) {
        double d = 1.0 + A[4 * j];
        for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
        if (!(d > 0.0)) return false;
        L[j][j] = std::sqrt(d);
        for (int i = j + 1; i < 3; ++i) {
            double s = A[3 * i + j];
            for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
            L[i][j] = s / L[j][j];
        }
    }
    double z[3];
    for (int i = 0; i < 3; ++i) {
        double s = r[i];
        for (int k = 0; k < i; ++k) s -= L[i][k] * z[k];
        z[i] = s / L[i][i];
    }
    for (int i = 2; i >= 0; --i) {
        double s = z[i];
        for (int k = i + 1; k < 3; ++k) s -= L[k][i] * y[k];
        y[i] = s / L[i][i];
    }
    return std::isfinite(y[0]) && std::isfinite(y[1]) && std::isfinite(y[2]);
}

double dist3(const double a[3], const double b[3])
{
    const double d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2];
    return std::sqrt(d0 * d0 + d1 * d1 + d2 * d2);
}

void store_state(double *traj, int32_t k, const double x[3], const double v[3])
{
    if (!traj) return;
    for (int i = 0; i < 3; ++i) {
        traj[6 * (size_t)k + i] = x[i];
        traj[6 * (size_t)k + 3 + i] = v[i];
    }
}

rmpc_status check_rollout(const rmpc_rollout_params *rp)
{
    if (!finite3(rp->goal)) return fail(RMPC_E_INVALID, "goal not finite");
    if (!(rp->alpha > 0.0) || !(rp->beta > 0.0) || !(rp->dt > 0.0) || !std::isfinite(rp->alpha) ||
        !std::isfinite(rp->beta) || !std::isfinite(rp->dt) || rp->max_steps < 0 || !(rp->goal_tol >= 0.0) ||
        !std::isfinite(rp->goal_tol) || !(rp->ray_weight >= 0.0) || !std::isfinite(rp->ray_weight) ||
        rp->smooth_every < 1)
        return fail(RMPC_E_INVALID, "rollout parameters out of range");
    return RMPC_OK;
}

// One flight's state between steps.
struct Flight {
    double x[3], v[3];
    double anchor[3];           // the last sampled state (smoothness)
    double prev[3];             // the last non-zero sampled displacement
    double path = 0.0, smooth_sum = 0.0;
    int64_t n_pairs = 0;
    int32_t k = 0;              // steps taken
    bool have_prev = false;
    bool done = false;
    uint32_t status = RMPC_ROLLOUT_TIMEOUT;

    void begin(const double x0[3], const double v0[3], double *traj)
    {
        std::memcpy(x, x0, sizeof x);
        std::memcpy(v, v0, sizeof v);
        std::memcpy(anchor, x0, sizeof anchor);
        store_state(traj, 0, x, v);
    }

    // Checks before the query of step k; true when the flight ends here.
    bool ends_before_query(const rmpc_rollout_params &rp)
    {
        if (k >= rp.max_steps) {
            done = true;        // TIMEOUT unless the last state is within goal_tol (finish)
        } else if (dist3(x, rp.goal) <= rp.goal_tol) {
            status = RMPC_ROLLOUT_GOAL;
            done = true;
        }
        return done;
    }

    void end(uint32_t st)
    {
        status = st;
        done = true;
    }

    // The step from the query's result: collision test, attractor, solve, integration, path
    // measures.  q.A, q.b are the query's sums.
    rmpc_status step(const rmpc_rollout_params &rp, double c, const rmpc_result &q, double *traj)
    {
        if (q.flags & RMPC_Q_IN_COLLISION) {
            end(RMPC_ROLLOUT_COLLISION);
            return RMPC_OK;
        }
        // f_a = alpha s(goal - x) - beta v (Eq. 3), metric I; a = (I + w A)^-1 (f_a + w b) (Eq. 1)
        double u[3], s[3], r[3], a[3], wA[9];
        for (int i = 0; i < 3; ++i) u[i] = rp.goal[i] - x[i];
        soft_normalize(u, c, s);
        for (int i = 0; i < 3; ++i) r[i] = rp.alpha * s[i] - rp.beta * v[i] + rp.ray_weight * q.b[i];
        for (int i = 0; i < 9; ++i) wA[i] = rp.ray_weight * q.A[i];
        if (!solve_identity_plus(wA, r, a)) return fail(RMPC_E_HIP, "metric sum is not positive semi-definite");
        double len2 = 0.0;
        for (int i = 0; i < 3; ++i) {
            v[i] += a[i] * rp.dt;
            const double xn = x[i] + v[i] * rp.dt;
            len2 += (xn - x[i]) * (xn - x[i]);
            x[i] = xn;
        }
        ++k;
        store_state(traj, k, x, v);
        path += std::sqrt(len2);
        if (k % rp.smooth_every == 0) {
            double seg[3];
            for (int i = 0; i < 3; ++i) seg[i] = x[i] - anchor[i];
            std::memcpy(anchor, x, sizeof anchor);
            const double len = std::sqrt(seg[0] * seg[0] + seg[1] * seg[1] + seg[2] * seg[2]);
            if (len > 0.0) {
                if (have_prev) {
                    const double pl = std::sqrt(prev[0] * prev[0] + prev[1] * prev[1] + prev[2] * prev[2]);
                    double cs = (prev[0] * seg[0] + prev[1] * seg[1] + prev[2] * seg[2]) / (pl * len);
                    cs = cs > 1.0 ? 1.0 : (cs < -1.0 ? -1.0 : cs);
                    smooth_sum += 1.0 - std::acos(cs) / kPi;
                    ++n_pairs;
                }
                std::memcpy(prev, seg, sizeof prev);
                have_prev = true;
            }
        }
        return RMPC_OK;
    }

    void finish(const rmpc_rollout_params &rp, rmpc_rollout_result *out) const
    {
        uint32_t st = status;
        if (st == RMPC_ROLLOUT_TIMEOUT && dist3(x, rp.goal) <= rp.goal_tol) st = RMPC_ROLLOUT_GOAL;
        out->status = st;
        out->n_steps = k;
        out->smoothness = n_pairs > 0 ? smooth_sum / (double)n_pairs : 1.0;
        out->path_length_m = path;
        std::memcpy(out->x, x, sizeof x);
        std::memcpy(out->v, v, sizeof v);
    }
};

}  // namespace

extern "C" {

rmpc_status rmpc_rollout(rmpc_ctx *ctx, int32_t map_id, const double x0[3], const double v0[3], int32_t n_rays,
                         const rmpc_params *params, const rmpc_rollout_params *rp, void *hip_stream,
                         double *traj_host, rmpc_rollout_result *out)
{
    if (!ctx || !params || !rp || !out) return fail(RMPC_E_INVALID, "NULL argument");
    if (!finite3(x0) || !finite3(v0)) return fail(RMPC_E_INVALID, "state not finite");
    if (rmpc_status st = check_rollout(rp)) return st;
    Flight F;
    F.begin(x0, v0, traj_host);
    while (!F.ends_before_query(*rp)) {
        rmpc_result q;
        const rmpc_status st = rmpc_query(ctx, map_id, F.x, F.v, n_rays, params, hip_stream, &q);
        if (st == RMPC_E_OUT_OF_BOUNDS) {
            F.end(RMPC_ROLLOUT_LEFT_GRID);
            break;
        }
        if (st != RMPC_OK) return st;
        if (rmpc_status e = F.step(*rp, params->c, q, traj_host)) return e;
    }
    F.finish(*rp, out);
    return RMPC_OK;
}

rmpc_status rmpc_rollout_batch(rmpc_ctx *ctx, const rmpc_flight *flights, int32_t n, const rmpc_params *params,
                               void *hip_stream, rmpc_rollout_result *out)
{
    if (!ctx || !flights || !params || !out) return fail(RMPC_E_INVALID, "NULL argument");
    if (n < 1) return fail(RMPC_E_INVALID, "n must be >= 1");
    if (rmpc_status st = rmpc_host::check_params(params)) return st;
    std::vector<const rmpc_host::MapEntry *> maps((size_t)n);
    for (int32_t i = 0; i < n; ++i) {
        const rmpc_flight &f = flights[i];
        const std::string where = "flight " + std::to_string(i) + ": ";
        auto it = ctx->maps.find(f.map_id);
        if (it == ctx->maps.end()) return fail(RMPC_E_NOMAP, where + "unknown map id");
        if (f.n_rays < 1 || f.n_rays > RMPC_MAX_RAYS) return fail(RMPC_E_INVALID, where + "n_rays out of [1, 65536]");
        if (!finite3(f.x0) || !finite3(f.v0)) return fail(RMPC_E_INVALID, where + "state not finite");
        if (rmpc_status st = check_rollout(&f.rp)) {
            rmpc_host::g_last_error = where + rmpc_host::g_last_error;
            return st;
        }
        maps[(size_t)i] = &it->second;
    }
    std::vector<Flight> F((size_t)n);
    for (int32_t i = 0; i < n; ++i) F[(size_t)i].begin(flights[i].x0, flights[i].v0, nullptr);
    std::vector<int32_t> live;
    std::vector<rmpc_query_desc> q;
    std::vector<rmpc_result> res;
    live.reserve((size_t)n);
    q.reserve((size_t)n);
    for (;;) {
        live.clear();
        q.clear();
        for (int32_t i = 0; i < n; ++i) {
            Flight &f = F[(size_t)i];
            if (f.done || f.ends_before_query(flights[i].rp)) continue;
            // the bounds test rmpc_query applies (dense: inside the grid; sparse: within reach)
            const rmpc_host::MapEntry &me = *maps[(size_t)i];
            float g[3];
            const bool inside = me.sparse ? rmpc_host::sparse_position_ok(me.desc, f.x, params->max_range_m / me.desc.voxel_m)
                                          : rmpc_host::grid_coords(me.desc, f.x, g);
            if (!inside) {
                f.end(RMPC_ROLLOUT_LEFT_GRID);
                continue;
            }
            rmpc_query_desc d;
            std::memset(&d, 0, sizeof d);
            d.kind = RMPC_KIND_MAP;
            d.map_id = flights[i].map_id;
            d.n = flights[i].n_rays;
            std::memcpy(d.x, f.x, sizeof d.x);
            std::memcpy(d.v, f.v, sizeof d.v);
            q.push_back(d);
            live.push_back(i);
        }
        if (live.empty()) break;
        res.resize(q.size());
        if (rmpc_status st = rmpc_query_batch(ctx, q.data(), (int32_t)q.size(), params, nullptr, hip_stream,
                                              res.data()))
            return st;
        for (size_t j = 0; j < live.size(); ++j) {
            const int32_t i = live[j];
            if (rmpc_status st = F[(size_t)i].step(flights[i].rp, params->c, res[j], nullptr)) return st;
        }
    }
    for (int32_t i = 0; i < n; ++i) F[(size_t)i].finish(flights[i].rp, &out[i]);
    return RMPC_OK;
}

}  // extern "C"
