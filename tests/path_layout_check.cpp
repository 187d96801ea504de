// CPU check of the tree factorisation tables (tree_layout.hpp): for many
// trees, build the elimination schedule and the path-pair layout the way
// robot upload does, then carry out on the CPU, in FP64 and lane by lane, the
// elimination the one-problem-per-wavefront kernel performs with them
// (partial rows per (joint, EE path) lane, one pivot per path and step, merge
// phases, back substitution by depth) on a random tree-structured system,
// and compare the step with a dense Gaussian elimination of the same system.
// Also checks structural properties of the tables.  Prints one line per
// failure and a summary; exit status 1 on any failure.
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "tree_layout.hpp"

using namespace pk;

static int failures = 0;
#define CHECK(c, ...)                                  \
    do {                                               \
        if (!(c)) {                                    \
            ++failures;                                \
            printf("FAIL %s: ", #c);                   \
            printf(__VA_ARGS__);                       \
            printf("\n");                              \
        }                                              \
    } while (0)

// The fields robot upload fills before the two table builders run.
static RobotC *make_robot(const std::vector<int> &parent, const std::vector<int> &ee)
{
    RobotC *R = new RobotC;
    memset(R, 0, sizeof *R);
    R->n = (int)parent.size();
    R->m = (int)ee.size();
    for (int j = 0; j < R->n; ++j) {
        const int par = parent[j];
        R->j[j].parent = par;
        R->j[j].depth = par < 0 ? 0 : R->j[par].depth + 1;
        if (R->j[j].depth > R->max_depth) R->max_depth = R->j[j].depth;
        R->janc[j] = par < 0 ? 0 : (R->janc[par] | (1ull << par));
        for (int d = 0; d < R->j[j].depth; ++d) R->anc_at[j][d] = R->anc_at[par][d];
        R->anc_at[j][R->j[j].depth] = (uint8_t)j;
    }
    build_step_schedule(*R);
    for (int k = 0; k < R->m; ++k) {
        R->e[k].joint = ee[k];
        uint64_t mask = 0;
        for (int a = ee[k]; a >= 0; a = parent[a]) mask |= 1ull << a;
        R->anc[k] = mask;
    }
    build_path_layout(*R);
    return R;
}

// Structure of the tables: lanes, copies, ancestors, one pivot per path and
// step, no update reaching a non-owner copy at or after its merge.
static void check_tables(const RobotC &R, int id)
{
    const PathC &P = R.path;
    const int L = P.lanes;
    std::vector<int> copies(R.n, 0);
    for (int l = 0; l < L; ++l) {
        const int j = P.joint[l], k = P.group[l], dep = R.j[j].depth;
        ++copies[j];
        CHECK(P.joint[P.owner[l]] == j, "tree %d lane %d owner holds another joint", id, l);
        if (k < 0) {
            CHECK(P.owner[l] == l, "tree %d lane %d: a joint on no path has one lane", id, l);
            continue;
        }
        CHECK((R.anc[k] >> j) & 1ull, "tree %d lane %d: joint %d not on path %d", id, l, j, k);
        for (int d = 0; d <= dep; ++d) {
            const int a = P.anc[l][d];
            CHECK(P.group[a] == k && P.joint[a] == R.anc_at[j][d], "tree %d lane %d depth %d", id, l, d);
        }
        for (int b = 0; b < 4; ++b) {
            const int a = (int)((P.jump[l] >> (8 * b)) & 0xffu), d = dep - (1 << b);
            CHECK(a == (d >= 0 ? P.anc[l][d] : l), "tree %d lane %d jump %d", id, l, b);
        }
        // updates only from pivots of this path below the joint, and none at
        // or after a non-owner copy's merge
        const bool owner = P.owner[l] == l;
        const int ms = owner ? 0 : P.merge_step[P.owner[l]];
        for (int s = 0; s < R.nstep; ++s) {
            if (!((P.upd[l] >> s) & 1ull)) continue;
            if (!owner) CHECK(ms != PK_PATH_NONE && s < ms, "tree %d lane %d update at %d after merge %d", id, l, s, ms);
        }
    }
    for (int j = 0; j < R.n; ++j) CHECK(copies[j] >= 1, "tree %d joint %d has no lane", id, j);
    for (int s = 0; s < R.nstep; ++s) {
        int per_group[PK_MAX_EES] = {0};
        for (int l = 0; l < L; ++l)
            if (P.owner[l] == l && P.group[l] >= 0 && R.step_of[P.joint[l]] == s) ++per_group[P.group[l]];
        for (int k = 0; k < R.m; ++k) CHECK(per_group[k] <= 1, "tree %d step %d: path %d owns %d pivots", id, s, k, per_group[k]);
    }
}

constexpr int DM = PK_PATH_MAX_DEPTH;

// The kernel's elimination on lanes, FP64, against a dense solve.
static double solve_check(const RobotC &R, std::mt19937 &rng, double lam)
{
    const PathC &P = R.path;
    const int n = R.n, m = R.m, L = 64;
    std::normal_distribution<double> N01;
    std::vector<double> J(m * 6 * n, 0.0), res(m * 6), extra(n);
    for (int k = 0; k < m; ++k)
        for (int u = 0; u < 6; ++u) {
            res[k * 6 + u] = N01(rng);
            for (int j = 0; j < n; ++j)
                if ((R.anc[k] >> j) & 1ull) J[(k * 6 + u) * n + j] = N01(rng);
        }
    for (int j = 0; j < n; ++j) extra[j] = 0.1 * std::fabs(N01(rng));   // limit and rest rows
    // dense (A + lam diag(max(A_jj, 1e-6))) x = -g by Gaussian elimination
    std::vector<double> A(n * n, 0.0), g(n, 0.0);
    for (int k = 0; k < m; ++k)
        for (int u = 0; u < 6; ++u)
            for (int i = 0; i < n; ++i) {
                g[i] += J[(k * 6 + u) * n + i] * res[k * 6 + u];
                for (int j = 0; j < n; ++j) A[i * n + j] += J[(k * 6 + u) * n + i] * J[(k * 6 + u) * n + j];
            }
    for (int j = 0; j < n; ++j) A[j * n + j] += extra[j];
    std::vector<double> M(A), x(n);
    for (int j = 0; j < n; ++j) {
        M[j * n + j] += lam * std::fmax(A[j * n + j], 1e-6);
        x[j] = -g[j];
    }
    for (int c = 0; c < n; ++c)
        for (int r = c + 1; r < n; ++r) {
            const double f = M[r * n + c] / M[c * n + c];
            for (int q = c; q < n; ++q) M[r * n + q] -= f * M[c * n + q];
            x[r] -= f * x[c];
        }
    for (int c = n - 1; c >= 0; --c) {
        for (int q = c + 1; q < n; ++q) x[c] -= M[c * n + q] * x[q];
        x[c] /= M[c * n + c];
    }
    // lanes: partial rows, partial diagonals, right-hand sides
    auto lj = [&](int l) { return l < P.lanes ? (int)P.joint[l] : -1; };
    auto lg = [&](int l) { return l < P.lanes ? (int)P.group[l] : -1; };
    auto ldep = [&](int l) { return l < P.lanes ? R.j[P.joint[l]].depth : -1; };
    auto lown = [&](int l) { return l < P.lanes && P.owner[l] == l; };
    auto lcopy = [&](int l, int c) { return l < P.lanes ? (int)P.copies[l][c] : (int)PK_PATH_NONE; };
    std::vector<std::array<double, DM>> r(L);
    std::vector<double> dgu(L, 0.0), gl(L, 0.0), dfull(L), dg(L), b(L), xl(L, 0.0), s(L, 0.0);
    for (int l = 0; l < L; ++l) {
        r[l].fill(0.0);
        const int j = lj(l), k = lg(l);
        if (k >= 0) {
            for (int d = 0; d <= ldep(l); ++d) {
                const int a = P.joint[P.anc[l][d]];
                double t = 0.0;
                for (int u = 0; u < 6; ++u) t += J[(k * 6 + u) * n + j] * J[(k * 6 + u) * n + a];
                if (d < ldep(l)) r[l][d] = t; else dgu[l] = t;
            }
            for (int u = 0; u < 6; ++u) gl[l] += J[(k * 6 + u) * n + j] * res[k * 6 + u];
        }
        if (lown(l)) dgu[l] += extra[j], gl[l] += 0.0;
    }
    for (int l = 0; l < L; ++l) {
        dfull[l] = dgu[l];
        if (lown(l))
            for (int c = 0; c < P.ncopy; ++c)
                if (lcopy(l, c) != PK_PATH_NONE) dfull[l] += dgu[lcopy(l, c)];
    }
    for (int l = 0; l < L; ++l) {
        dg[l] = dgu[l] + (lown(l) ? lam * std::fmax(dfull[l], 1e-6) : 0.0);
        b[l] = lj(l) >= 0 ? -gl[l] : 0.0;
    }
    std::vector<std::array<double, DM + 2>> slot(PK_MAX_EES);
    for (int st = 0; st < R.nstep; ++st) {
        const int pdep = P.step_info[st] & 0xff, mdep = (P.step_info[st] >> 8) & 0xff;
        if (mdep > 0) {
            const auto r0 = r;
            const auto dg0 = dg, b0 = b;
            for (int l = 0; l < L; ++l)
                if (lown(l) && P.merge_step[l] == st)
                    for (int c = 0; c < P.ncopy; ++c) {
                        const int cl = lcopy(l, c);
                        if (cl == PK_PATH_NONE) continue;
                        for (int d = 0; d + 1 < mdep; ++d) r[l][d] += r0[cl][d];
                        dg[l] += dg0[cl];
                        b[l] += b0[cl];
                    }
        }
        for (int l = 0; l < L; ++l)
            if (lown(l) && R.step_of[lj(l)] == st) {
                CHECK(dg[l] > 0.0, "pivot of lane %d at step %d is %g", l, st, dg[l]);
                if (lg(l) >= 0) {
                    auto &sl = slot[lg(l)];
                    for (int d = 0; d < DM; ++d) sl[d] = r[l][d];
                    sl[DM] = dg[l];
                    sl[DM + 1] = b[l];
                }
            }
        for (int l = 0; l < P.lanes; ++l)
            if ((P.upd[l] >> st) & 1ull) {
                const auto &sk = slot[lg(l)];
                const double c = sk[ldep(l)] / sk[DM];
                for (int i = 0; i < DM / 4; ++i)
                    if (4 * i < pdep)
                        for (int d = 4 * i; d < 4 * i + 4; ++d) r[l][d] -= c * sk[d];
                dg[l] -= c * sk[ldep(l)];
                b[l] -= c * sk[DM + 1];
            }
    }
    for (int D = 0; D <= R.max_depth; ++D) {
        for (int l = 0; l < L; ++l)
            if (lown(l) && ldep(l) == D) xl[l] = (b[l] - s[l]) / dg[l];
        if ((P.copy_depths >> D) & 1u) {
            const auto x0 = xl;
            for (int l = 0; l < L; ++l)
                if (ldep(l) == D) xl[l] = x0[l < P.lanes ? P.owner[l] : l];
        }
        const auto x1 = xl;
        for (int l = 0; l < L; ++l)
            if (ldep(l) > D) s[l] += r[l][D] * x1[l < P.lanes ? P.anc[l][D] : l];
    }
    double err = 0.0, mx = 0.0;
    for (int l = 0; l < L; ++l)
        if (lj(l) >= 0) {
            err = std::fmax(err, std::fabs(xl[l] - x[lj(l)]));
            mx = std::fmax(mx, std::fabs(x[lj(l)]));
        }
    return err / (mx + 1e-300);
}

int main()
{
    std::mt19937 rng(20250503);
    std::vector<std::pair<std::vector<int>, std::vector<int>>> trees;
    {   // torso of 6 and 4 branches of 7, an EE at each branch tip
        std::vector<int> p, e;
        for (int j = 0; j < 6; ++j) p.push_back(j - 1);
        for (int c = 0; c < 4; ++c)
            for (int i = 0; i < 7; ++i) {
                const int j = 6 + c * 7 + i;
                p.push_back(i == 0 ? 5 : j - 1);
                if (i == 6) e.push_back(j);
            }
        trees.push_back({p, e});
    }
    {   // 4 fingers of 4 from the base
        std::vector<int> p, e;
        for (int c = 0; c < 4; ++c)
            for (int i = 0; i < 4; ++i) {
                const int j = c * 4 + i;
                p.push_back(i == 0 ? -1 : j - 1);
                if (i == 3) e.push_back(j);
            }
        trees.push_back({p, e});
    }
    trees.push_back({{-1, 0, 1, 2, 3, 4, 5}, {6}});              // chain
    trees.push_back({{-1, 0, 1, 2, 3, 4, 5}, {6, 3}});           // an EE on another EE's path
    trees.push_back({{-1, 0, 1, 2, 3, 4, 5}, {6, 6}});           // two EEs on one joint
    trees.push_back({{-1, 0, 1, 1, 3, 2, 0, 6}, {5, 4}});        // joints 6, 7 on no EE path
    {   // 20 leaves under one root (a height level split into two steps), 8 EEs
        std::vector<int> p{-1}, e;
        for (int j = 1; j <= 20; ++j) p.push_back(0);
        for (int k = 0; k < 8; ++k) e.push_back(1 + 2 * k);
        trees.push_back({p, e});
    }
    std::uniform_int_distribution<int> U(0, 1 << 30);
    for (int t = 0; t < 300; ++t) {
        const int n = 2 + U(rng) % 60;
        std::vector<int> p(n);
        p[0] = -1;
        for (int j = 1; j < n; ++j) {
            const int lo = j > 6 ? j - 6 : 0;
            p[j] = (U(rng) % 5 == 0) ? -1 : lo + U(rng) % (j - lo);
        }
        std::vector<int> e(1 + U(rng) % 8);
        for (auto &k : e) k = U(rng) % n;
        trees.push_back({p, e});
    }
    int checked = 0, skipped = 0, shared = 0;
    double worst = 0.0;
    for (size_t id = 0; id < trees.size(); ++id) {
        RobotC *R = make_robot(trees[id].first, trees[id].second);
        if (!R->path.ok) {
            ++skipped;
            CHECK(id >= 7, "hand-written tree %zu does not fit the layout", id);
            delete R;
            continue;
        }
        check_tables(*R, (int)id);
        shared += R->path.ncopy > 0;
        for (double lam : {1e-6, 1e-3, 1.0}) {
            const double e = solve_check(*R, rng, lam);
            worst = std::fmax(worst, e);
            CHECK(e <= 1e-9, "tree %zu (n=%d, m=%d, lanes=%d) lambda %g: relative error %.3g", id, R->n,
                  R->m, R->path.lanes, lam, e);
        }
        ++checked;
        delete R;
    }
    RobotC *T = make_robot(trees[0].first, trees[0].second);
    CHECK(T->path.lanes == 52 && T->path.ncopy == 3 && T->nstep == 13, "torso tree: %d lanes, %d copies, %d steps",
          T->path.lanes, T->path.ncopy, T->nstep);
    delete T;
    printf("checked %d trees (%d with shared joints, %d beyond the layout), worst relative error %.3g, %d failures\n",
           checked, shared, skipped, worst, failures);
    return failures ? 1 : 0;
}
