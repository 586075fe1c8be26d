// rollout.hip -- closed-loop rollout (Sec. III-A Eq. 1 with the goal attractor of Sec. III-B
// Eqs. 2-3): every state's ray policy comes from one rmpc_query launch; the attractor, the 3x3
// solve and the integration are a few float64 operations on the host around it.

#include <cmath>
#include <cstring>

#include "rmpc_host.h"

using rmpc_host::fail;
using rmpc_host::finite3;

namespace {

constexpr double kPi = 3.14159265358979323846;

// Eq. 3: s(u) = u / (|u| + c log(1 + exp(-2 c |u|))).
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

}  // namespace

extern "C" {

rmpc_status rmpc_rollout(rmpc_ctx *ctx, int32_t map_id, const double x0[3], const double v0[3], int32_t n_rays,
                         const rmpc_params *params, const rmpc_rollout_params *rp, void *hip_stream,
                         double *traj_host, rmpc_rollout_result *out)
{
    if (!ctx || !params || !rp || !out) return fail(RMPC_E_INVALID, "NULL argument");
    if (!finite3(x0) || !finite3(v0) || !finite3(rp->goal)) return fail(RMPC_E_INVALID, "state or goal not finite");
    if (!(rp->alpha > 0.0) || !(rp->beta > 0.0) || !(rp->dt > 0.0) || !std::isfinite(rp->alpha) ||
        !std::isfinite(rp->beta) || !std::isfinite(rp->dt) || rp->max_steps < 0 || !(rp->goal_tol >= 0.0) ||
        !std::isfinite(rp->goal_tol) || !(rp->ray_weight >= 0.0) || !std::isfinite(rp->ray_weight))
        return fail(RMPC_E_INVALID, "rollout parameters out of range");
    double x[3], v[3];
    std::memcpy(x, x0, sizeof x);
    std::memcpy(v, v0, sizeof v);
    store_state(traj_host, 0, x, v);
    uint32_t status = RMPC_ROLLOUT_TIMEOUT;
    int32_t k = 0;
    double path = 0.0, smooth_sum = 0.0, prev[3] = {0.0, 0.0, 0.0};
    int64_t n_pairs = 0;
    bool have_prev = false;
    for (; k < rp->max_steps; ++k) {
        if (dist3(x, rp->goal) <= rp->goal_tol) {
            status = RMPC_ROLLOUT_GOAL;
            break;
        }
        rmpc_result q;
        const rmpc_status st = rmpc_query(ctx, map_id, x, v, n_rays, params, hip_stream, &q);
        if (st == RMPC_E_OUT_OF_BOUNDS) {
            status = RMPC_ROLLOUT_LEFT_GRID;
            break;
        }
        if (st != RMPC_OK) return st;
        if (q.flags & RMPC_Q_IN_COLLISION) {
            status = RMPC_ROLLOUT_COLLISION;
            break;
        }
        // f_a = alpha s(goal - x) - beta v (Eq. 2), metric I; a = (I + w A)^-1 (f_a + w b) (Eq. 1)
        double u[3], s[3], r[3], a[3], wA[9];
        for (int i = 0; i < 3; ++i) u[i] = rp->goal[i] - x[i];
        soft_normalize(u, params->c, s);
        for (int i = 0; i < 3; ++i) r[i] = rp->alpha * s[i] - rp->beta * v[i] + rp->ray_weight * q.b[i];
        for (int i = 0; i < 9; ++i) wA[i] = rp->ray_weight * q.A[i];
        if (!solve_identity_plus(wA, r, a)) return fail(RMPC_E_HIP, "metric sum is not positive semi-definite");
        double seg[3];
        for (int i = 0; i < 3; ++i) {
            v[i] += a[i] * rp->dt;
            const double xn = x[i] + v[i] * rp->dt;
            seg[i] = xn - x[i];
            x[i] = xn;
        }
        store_state(traj_host, k + 1, x, v);
        const double len = std::sqrt(seg[0] * seg[0] + seg[1] * seg[1] + seg[2] * seg[2]);
        path += len;
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
    if (status == RMPC_ROLLOUT_TIMEOUT && dist3(x, rp->goal) <= rp->goal_tol) status = RMPC_ROLLOUT_GOAL;
    out->status = status;
    out->n_steps = k;
    out->smoothness = n_pairs > 0 ? smooth_sum / (double)n_pairs : 1.0;
    out->path_length_m = path;
    std::memcpy(out->x, x, sizeof x);
    std::memcpy(out->v, v, sizeof v);
    return RMPC_OK;
}

}  // extern "C"
