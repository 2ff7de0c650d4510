// Internal declarations of the colour-coding library (host side).
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/ccgpu.h"

namespace ccg {

constexpr int kMaxPattern = 16;  // n_F limit of a decomposition
constexpr int kMaxColours = 16;    // k limit of a colouring and of every DP run
constexpr int kDenseColours = 12;  // k limit of the dense 2^k colour-set accumulators
constexpr int kMaxBag = 4;       // bag size limit of the device kernels (width <= 3)

enum NodeType { LEAF = 0, INTRO = 1, FORGET = 2, JOIN = 3 };

struct TdNode {
    int type;
    int u;       // vertex of a leaf / introduce / forget node, -1 for a join
    int c0, c1;  // children (post-order indices), -1 if absent
    uint32_t bag;
};

// A pattern F with its nice tree decomposition (Sec. 1.2, Sec. 3).
struct Decomp {
    int n = 0;
    std::vector<std::pair<int, int>> edges;
    uint32_t adj[32] = {0};
    int width = 0;
    std::vector<TdNode> nodes;  // post-order, root last
};

// Device plan: one step per DP table the device materialises.
enum StepKind {
    S_LEAF,         // (bid, u) for every vertex passing the degree mask
    S_INTRO_PUSH,   // u inserted at column `pos`, candidates from the anchor's row
    S_INTRO_PULL,   // u inserted at column 0, child grouped by its column 0 (the anchor)
    S_FORGET_LAST,  // drop the last column and add equal (prefix, colour set) keys
    S_JOIN,         // merge two tables with identical column order
    S_RESORT,       // permute the columns and re-sort (no reduction)
};

struct Step {
    StepKind kind;
    int node = -1;         // TD node whose table this step yields (-1: auxiliary)
    int in0 = -1, in1 = -1;  // input steps
    int u = -1;            // pattern vertex of the step
    int b_in = 0, b_out = 0;
    int cols[kMaxBag] = {-1, -1, -1, -1};  // pattern vertex held by each output column
    int pos = 0;           // introduce: output column of u
    int anchor = -1;       // introduce: child column whose image gives the candidates (-1: all of V(G))
    int nchk = 0;
    int chk[kMaxBag] = {0};  // introduce: further child columns adjacent to u in F
    int degF = 0;          // deg_F(u)
    int perm[kMaxBag] = {0};  // resort: output column j <- input column perm[j]
};

struct Plan {
    std::vector<Step> steps;
    int root_child = -1;  // step whose table is the node below the root (bag {0})
    int max_bag = 0;
};

// planner.cpp
int build_decomposition(int nF, const std::vector<std::pair<int, int>>& edges, Decomp* out,
                        std::string* err);
int validate_decomposition(const Decomp& d, std::string* err);
int make_plan(const Decomp& d, Plan* plan, std::string* err);
std::string describe_plan(const Decomp& d, const Plan& plan);

// errors
void set_error(const std::string& msg);

}  // namespace ccg
