// Host planner: exact-width tree decomposition of the pattern (Sec. 3), its
// nice form (Sec. 1.2), and the device plan with one column order per table.
//
// Column orders.  A DP table is kept sorted by the key (colouring index,
// images of the bag in the table's column order, colour set).  A forget node
// then only streams over runs of equal prefixes when the forgotten vertex is
// the LAST column, and a join node merges its children when both use the
// same order.  Both hold by construction when every table lists its bag in
// order of decreasing "forget time" (the post-order index of the node that
// forgets the vertex): the next vertex to be forgotten is always last, and
// the two children of a join share their forget times.  An introduce node
// must then insert its vertex u at the column its forget time dictates; the
// planner uses
//   - a push step (candidates from the image of a bag neighbour of u that
//     sits before the insertion column, so equal prefixes stay contiguous),
//   - a pull step (insertion at column 0, the child's column 0 being a
//     neighbour of u: the output is produced per image of u by gathering the
//     child's runs of that neighbour's images), or
//   - a push at the end followed by a re-sort when neither applies,
// and a full scan of V(G) when u has no neighbour in the bag (Sec. 3.2, last
// paragraph of "Mapping Expansion Optimizations").
#include <algorithm>
#include <cstring>
#include <functional>
#include <numeric>
#include <random>

#include "internal.h"

namespace ccg {

namespace {

int popcount32(uint32_t x) { return __builtin_popcount(x); }

// Vertices outside `elim` and v reachable from v through vertices of `elim`:
// v's neighbourhood in the graph filled by eliminating `elim` first.
uint32_t fill_neighbours(const uint32_t* adj, uint32_t elim, int v) {
    uint32_t visited = 1u << v, frontier = 1u << v, result = 0;
    while (frontier) {
        uint32_t nb = 0;
        for (uint32_t m = frontier; m; m &= m - 1) nb |= adj[__builtin_ctz(m)];
        nb &= ~visited;
        visited |= nb;
        result |= nb & ~elim;  // reached outer vertices are not expanded
        frontier = nb & elim;  // paths continue through eliminated vertices
    }
    return result;
}

// Minimum-width elimination order with vertex 0 last.  width_of[S] is the
// least possible maximum fill degree when exactly the vertices of S are
// eliminated first; the order is read back from the argmin table.  `rng`
// breaks ties between equally good choices (different valid optima).
int exact_order(int n, const uint32_t* adj, std::mt19937* rng, std::vector<int>* order) {
    const uint32_t others = ((n == 32) ? 0xFFFFFFFFu : ((1u << n) - 1u)) & ~1u;
    const size_t states = size_t(1) << n;
    std::vector<int8_t> width_of(states, 127);
    std::vector<int8_t> choice(states, -1);
    width_of[0] = -1;
    for (uint32_t S = 1; S < states; S++) {
        if (S & ~others) continue;
        int best = 127, nbest = 0;
        for (uint32_t m = S; m; m &= m - 1) {
            int v = __builtin_ctz(m);
            uint32_t before = S & ~(1u << v);
            int w = std::max<int>(width_of[before], popcount32(fill_neighbours(adj, before, v)));
            if (w < best) {
                best = w;
                choice[S] = int8_t(v);
                nbest = 1;
            } else if (w == best && rng) {
                // reservoir choice among ties
                nbest++;
                if ((*rng)() % nbest == 0) choice[S] = int8_t(v);
            }
        }
        width_of[S] = int8_t(best);
    }
    order->assign(n, 0);
    uint32_t S = others;
    for (int i = n - 2; i >= 0; i--) {
        (*order)[i] = choice[S];
        S &= ~(1u << choice[S]);
    }
    (*order)[n - 1] = 0;
    int width = std::max<int>(width_of[others], popcount32(fill_neighbours(adj, others, 0)));
    return std::max(width, 0);
}

struct NiceBuilder {
    const uint32_t* adj;
    std::vector<TdNode> nodes;
    std::mt19937* rng;

    int add(int type, int u, int c0, int c1, uint32_t bag) {
        nodes.push_back({type, u, c0, c1, bag});
        return int(nodes.size()) - 1;
    }

    // introduce the vertices of `target` missing from `bag`, anchored ones first
    int introduce_to(int top, uint32_t bag, uint32_t target) {
        uint32_t missing = target & ~bag;
        while (missing) {
            int pick = -1;
            std::vector<int> anchored;
            for (uint32_t m = missing; m; m &= m - 1) {
                int v = __builtin_ctz(m);
                if (adj[v] & bag) anchored.push_back(v);
            }
            if (!anchored.empty())
                pick = anchored[rng ? (*rng)() % anchored.size() : 0];
            else
                pick = __builtin_ctz(missing);
            bag |= 1u << pick;
            missing &= ~(1u << pick);
            top = add(INTRO, pick, top, -1, bag);
        }
        return top;
    }

    int forget_to(int top, uint32_t bag, uint32_t keep) {
        for (uint32_t m = bag & ~keep; m; m &= m - 1) {
            int v = __builtin_ctz(m);
            bag &= ~(1u << v);
            top = add(FORGET, v, top, -1, bag);
        }
        return top;
    }
};

}  // namespace

static int build_one(const Decomp& base, std::mt19937* rng, Decomp* out) {
    const int n = base.n;
    std::vector<int> order;
    int width = exact_order(n, base.adj, rng, &order);
    std::vector<int> pos(n);
    for (int i = 0; i < n; i++) pos[order[i]] = i;
    std::vector<uint32_t> bag(n);
    std::vector<int> parent(n, -1);
    uint32_t done = 0;
    for (int i = 0; i < n; i++) {
        int v = order[i];
        uint32_t q = fill_neighbours(base.adj, done, v);
        bag[v] = q | (1u << v);
        int first = -1;
        for (uint32_t m = q; m; m &= m - 1) {
            int w = __builtin_ctz(m);
            if (first < 0 || pos[w] < pos[first]) first = w;
        }
        parent[v] = first;
        done |= 1u << v;
    }
    for (int v = 1; v < n; v++)
        if (parent[v] < 0) parent[v] = 0;  // other components hang below vertex 0

    NiceBuilder nb{base.adj, {}, rng};
    // Branches are joined at the smallest bag they can share (the union of
    // their bags' intersections with the parent's bag); the parent's other
    // vertices are introduced once, after the join.  Join tables then key on
    // as few images as possible.
    std::function<int(int)> below = [&](int v) -> int {
        std::vector<std::pair<int, uint32_t>> branches;  // (top node, bag)
        for (int c = 0; c < n; c++) {
            if (c == v || parent[c] != v) continue;
            int top = below(c);
            top = nb.forget_to(top, bag[c], bag[v]);
            branches.push_back({top, bag[c] & bag[v]});
        }
        if (branches.empty()) {
            int top = nb.add(LEAF, v, -1, -1, 1u << v);
            return nb.introduce_to(top, 1u << v, bag[v]);
        }
        uint32_t common = 0;
        for (auto& b : branches) common |= b.second;
        if (common == 0) common = 1u << v;  // only fully forgotten branches: meet at {v}
        int top = -1;
        for (auto& b : branches) {
            int t = nb.introduce_to(b.first, b.second, common);
            top = top < 0 ? t : nb.add(JOIN, -1, top, t, common);
        }
        return nb.introduce_to(top, common, bag[v]);
    };
    int top = below(0);
    top = nb.forget_to(top, bag[0], 1u);  // bag[0] == {0}: nothing to do
    nb.add(FORGET, 0, top, -1, 0u);
    *out = base;
    out->width = width;
    out->nodes = std::move(nb.nodes);
    return CC_OK;
}

// ---------------------------------------------------------------------------
// Plan construction

namespace {

struct PlanScore {
    int full_scans = 0, resorts = 0, pulls = 0, bag_sum = 0;
    bool operator<(const PlanScore& o) const {
        if (full_scans != o.full_scans) return full_scans < o.full_scans;
        if (resorts != o.resorts) return resorts < o.resorts;
        return bag_sum < o.bag_sum;
    }
};

int plan_for(const Decomp& d, Plan* plan, PlanScore* score, std::string* err) {
    const int N = int(d.nodes.size());
    // forget time of each pattern vertex
    std::vector<int> ftime(d.n, -1);
    for (int i = 0; i < N; i++)
        if (d.nodes[i].type == FORGET) ftime[d.nodes[i].u] = i;
    for (int v = 0; v < d.n; v++)
        if (ftime[v] < 0) {
            if (err) *err = "pattern vertex is never forgotten";
            return CC_EINVAL;
        }
    auto ordered = [&](uint32_t bag, int* cols) {
        int b = 0;
        for (uint32_t m = bag; m; m &= m - 1) cols[b++] = __builtin_ctz(m);
        std::sort(cols, cols + b, [&](int a, int c) { return ftime[a] > ftime[c]; });
        return b;
    };
    plan->steps.clear();
    plan->max_bag = 0;
    *score = PlanScore();
    std::vector<int> step_of(N, -1);
    for (int i = 0; i < N; i++) {
        const TdNode& x = d.nodes[i];
        Step s;
        s.node = i;
        s.u = x.u;
        int cols[32];
        int b = ordered(x.bag, cols);
        if (b > kMaxBag) {
            if (err) *err = "bag larger than 4 (treewidth above 3)";
            return CC_ERANGE;
        }
        plan->max_bag = std::max(plan->max_bag, b);
        s.b_out = b;
        for (int j = 0; j < b; j++) s.cols[j] = cols[j];
        score->bag_sum += b;
        if (x.type == LEAF) {
            s.kind = S_LEAF;
            s.degF = popcount32(d.adj[x.u]);
        } else if (x.type == FORGET) {
            if (i == N - 1) {  // the root: counts are read from its child
                plan->root_child = step_of[x.c0];
                continue;
            }
            const Step& c = plan->steps[step_of[x.c0]];
            if (c.cols[c.b_out - 1] != x.u) {
                if (err) *err = "internal: forgotten vertex is not the last column";
                return CC_EINVAL;
            }
            s.kind = S_FORGET_LAST;
            s.in0 = step_of[x.c0];
            s.b_in = c.b_out;
        } else if (x.type == JOIN) {
            const Step& y = plan->steps[step_of[x.c0]];
            const Step& z = plan->steps[step_of[x.c1]];
            if (memcmp(y.cols, z.cols, sizeof y.cols) != 0 || memcmp(y.cols, s.cols, sizeof s.cols) != 0) {
                if (err) *err = "internal: join children disagree on column order";
                return CC_EINVAL;
            }
            s.kind = S_JOIN;
            s.in0 = step_of[x.c0];
            s.in1 = step_of[x.c1];
            s.b_in = b;
        } else {  // INTRO
            const Step& c = plan->steps[step_of[x.c0]];
            s.in0 = step_of[x.c0];
            s.b_in = c.b_out;
            s.degF = popcount32(d.adj[x.u]);
            int p = 0;
            while (s.cols[p] != x.u) p++;
            // child columns holding neighbours of u
            int nbr[kMaxBag], nn = 0;
            for (int j = 0; j < c.b_out; j++)
                if (d.adj[x.u] >> c.cols[j] & 1) nbr[nn++] = j;
            auto set_checks = [&](int anchor) {
                s.nchk = 0;
                for (int t = 0; t < nn; t++)
                    if (nbr[t] != anchor) s.chk[s.nchk++] = nbr[t];
            };
            int anchor_before = -1;
            for (int t = 0; t < nn; t++)
                if (nbr[t] < p) { anchor_before = nbr[t]; break; }
            if (nn == 0) {
                s.kind = S_INTRO_PUSH;
                s.pos = p;
                s.anchor = -1;
                s.nchk = 0;
                score->full_scans++;
            } else if (anchor_before >= 0) {
                s.kind = S_INTRO_PUSH;
                s.pos = p;
                s.anchor = anchor_before;
                set_checks(anchor_before);
            } else if (p == 0 && (d.adj[x.u] >> c.cols[0] & 1)) {
                s.kind = S_INTRO_PULL;
                s.pos = 0;
                s.anchor = 0;
                set_checks(0);
                score->pulls++;
            } else {
                // push at the end, then re-sort into the planned order
                Step t = s;
                t.kind = S_INTRO_PUSH;
                t.node = -1;
                t.pos = c.b_out;
                t.anchor = nbr[0];
                t.nchk = 0;
                for (int q = 1; q < nn; q++) t.chk[t.nchk++] = nbr[q];
                for (int j = 0; j < c.b_out; j++) t.cols[j] = c.cols[j];
                t.cols[c.b_out] = x.u;
                plan->steps.push_back(t);
                Step r;
                r.kind = S_RESORT;
                r.node = i;
                r.in0 = int(plan->steps.size()) - 1;
                r.u = x.u;
                r.b_in = b;
                r.b_out = b;
                for (int j = 0; j < b; j++) {
                    r.cols[j] = s.cols[j];
                    int q = 0;
                    while (t.cols[q] != s.cols[j]) q++;
                    r.perm[j] = q;
                }
                plan->steps.push_back(r);
                step_of[i] = int(plan->steps.size()) - 1;
                score->resorts++;
                continue;
            }
        }
        plan->steps.push_back(s);
        step_of[i] = int(plan->steps.size()) - 1;
    }
    if (plan->root_child < 0) {
        if (err) *err = "internal: no root";
        return CC_EINVAL;
    }
    return CC_OK;
}

}  // namespace

int build_decomposition(int nF, const std::vector<std::pair<int, int>>& edges, Decomp* out,
                        std::string* err) {
    if (nF < 1 || nF > kMaxPattern) {
        if (err) *err = "pattern size must be in [1, 16]";
        return CC_ERANGE;
    }
    Decomp base;
    base.n = nF;
    for (auto& e : edges) {
        if (e.first < 0 || e.second < 0 || e.first >= nF || e.second >= nF || e.first == e.second) {
            if (err) *err = "pattern edge out of range or a loop";
            return CC_EINVAL;
        }
        base.adj[e.first] |= 1u << e.second;
        base.adj[e.second] |= 1u << e.first;
    }
    for (int a = 0; a < nF; a++)
        for (uint32_t m = base.adj[a]; m; m &= m - 1) {
            int b = __builtin_ctz(m);
            if (a < b) base.edges.push_back({a, b});
        }
    // several optimal decompositions (ties broken at random, seeded), the
    // one whose plan needs the fewest full scans and re-sorts wins
    Decomp best;
    PlanScore best_score;
    bool have = false;
    for (int trial = 0; trial < 24; trial++) {
        std::mt19937 rng(0x5EED + trial);
        Decomp cand;
        build_one(base, trial == 0 ? nullptr : &rng, &cand);
        Plan p;
        PlanScore sc;
        std::string e2;
        if (plan_for(cand, &p, &sc, &e2) != CC_OK) continue;
        if (!have || sc < best_score) {
            best = cand;
            best_score = sc;
            have = true;
        }
    }
    if (!have) {
        if (err) *err = "no decomposition with bags of at most 4 vertices (treewidth > 3)";
        return CC_ERANGE;
    }
    *out = best;
    return validate_decomposition(*out, err);
}

int validate_decomposition(const Decomp& d, std::string* err) {
    auto fail = [&](const char* m) {
        if (err) *err = m;
        return CC_EINVAL;
    };
    const int N = int(d.nodes.size());
    if (N < 1) return fail("empty decomposition");
    const uint32_t all = (d.n == 32) ? 0xFFFFFFFFu : ((1u << d.n) - 1u);
    std::vector<int> up(N, -1);
    for (int i = 0; i < N; i++) {
        const TdNode& x = d.nodes[i];
        if (x.bag & ~all) return fail("bag holds a vertex outside the pattern");
        for (int c : {x.c0, x.c1}) {
            if (c < 0) continue;
            if (c >= i) return fail("nodes are not in post-order");
            if (up[c] >= 0) return fail("node with two parents");
            up[c] = i;
        }
        auto in_child = [&](int c, int v) { return (d.nodes[c].bag >> v & 1) != 0; };
        switch (x.type) {
            case LEAF:
                if (x.c0 >= 0 || x.c1 >= 0 || x.u < 0 || x.u >= d.n || x.bag != (1u << x.u))
                    return fail("bad leaf node");
                break;
            case INTRO:
                if (x.c0 < 0 || x.c1 >= 0 || x.u < 0 || x.u >= d.n || in_child(x.c0, x.u) ||
                    x.bag != (d.nodes[x.c0].bag | (1u << x.u)))
                    return fail("bad introduce node");
                break;
            case FORGET:
                if (x.c0 < 0 || x.c1 >= 0 || x.u < 0 || x.u >= d.n || !in_child(x.c0, x.u) ||
                    x.bag != (d.nodes[x.c0].bag & ~(1u << x.u)))
                    return fail("bad forget node");
                break;
            case JOIN:
                if (x.c0 < 0 || x.c1 < 0 || x.bag != d.nodes[x.c0].bag || x.bag != d.nodes[x.c1].bag)
                    return fail("bad join node");
                break;
            default:
                return fail("unknown node type");
        }
    }
    for (int i = 0; i + 1 < N; i++)
        if (up[i] < 0) return fail("node without parent");
    const TdNode& r = d.nodes[N - 1];
    if (r.bag != 0 || r.c0 < 0 || r.c1 >= 0) return fail("root must have an empty bag and one child");
    uint32_t seen = 0;
    for (const TdNode& x : d.nodes) seen |= x.bag;
    if (seen != all) return fail("a vertex is in no bag");
    for (auto& e : d.edges) {
        bool ok = false;
        for (const TdNode& x : d.nodes)
            if ((x.bag >> e.first & 1) && (x.bag >> e.second & 1)) ok = true;
        if (!ok) return fail("an edge is in no bag");
    }
    for (int v = 0; v < d.n; v++) {  // connectivity: one topmost node per vertex
        int tops = 0;
        for (int i = 0; i < N; i++)
            if ((d.nodes[i].bag >> v & 1) && (up[i] < 0 || !(d.nodes[up[i]].bag >> v & 1))) tops++;
        if (tops != 1) return fail("the nodes of a vertex are not connected");
    }
    return CC_OK;
}

std::string describe_plan(const Decomp& d, const Plan& plan) {
    static const char* names[] = {"leaf", "intro-push", "intro-pull", "forget-last", "join", "resort"};
    std::string out;
    char line[256];
    for (size_t i = 0; i < plan.steps.size(); i++) {
        const Step& s = plan.steps[i];
        std::string cols = "(";
        for (int j = 0; j < s.b_out; j++) cols += (j ? "," : "") + std::to_string(s.cols[j]);
        cols += ")";
        snprintf(line, sizeof line, "%2zu %-11s u=%-2d in=%d,%d node=%d cols=%s", i, names[s.kind], s.u, s.in0, s.in1,
                 s.node, cols.c_str());
        out += line;
        if (s.kind == S_INTRO_PUSH || s.kind == S_INTRO_PULL) {
            snprintf(line, sizeof line, " pos=%d anchor=%d checks=%d", s.pos, s.anchor, s.nchk);
            out += line;
        }
        out += "\n";
    }
    snprintf(line, sizeof line, "root <- step %d; width %d\n", plan.root_child, d.width);
    out += line;
    return out;
}

int make_plan(const Decomp& d, Plan* plan, std::string* err) {
    PlanScore sc;
    return plan_for(d, plan, &sc, err);
}

}  // namespace ccg
