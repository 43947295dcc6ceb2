// Greedy gate-fusion planner (host only).
//
// A block is opened at the first unassigned gate. Later unassigned gates are
// scanned in circuit order; a gate joins the block when its qubits (targets
// and controls) are disjoint from every qubit "blocked" so far and the union
// with the block's qubits has at most max_k members. A gate that cannot join
// blocks its qubits: no later gate touching them may be moved in front of
// it. Since a joining gate shares no qubit with any gate it overtakes, the
// two commute, and applying the blocks in order equals applying the gates in
// order.
//
// Rows far apart. A block whose targets include several qubits at or above
// far_lo has its 2^k amplitudes in rows 16 MiB or more apart that share their
// low address bits; such sweeps run up to 1.6x slower than blocks over nearby
// rows (the memory serves them from the same banks). A second plan is made in
// which a gate does not join a block when it would bring a second far qubit
// into it (it is skipped like a gate that does not fit, which keeps the order
// argument above intact; a block's first gate may bring more), and the plan
// with the lower estimated sweep time is kept: every block costs 1, 1.05,
// 1.10, 1.19 or 1.30 for 0..4 far qubits (the measured busy time of 30-qubit
// complex128 4-qubit sweeps relative to blocks without far qubits).
#include <algorithm>
#include <cstdint>
#include <vector>

#include "qs_internal.h"

namespace qs {

namespace {

int plan_greedy(int n_qubits, int n_gates, const int *k, const int *targets, const uint64_t *ctrl_mask,
                int max_k, Plan &out, int far_lo)
{
    out.block_of_gate.assign(size_t(n_gates), -1);
    out.block_gates.clear();
    out.block_qubits.clear();
    std::vector<uint64_t> gmask(static_cast<size_t>(n_gates));
    std::vector<size_t> toff(size_t(n_gates) + 1, 0);
    for (int g = 0; g < n_gates; ++g) toff[size_t(g) + 1] = toff[size_t(g)] + size_t(k[g]);
    for (int g = 0; g < n_gates; ++g) {
        uint64_t m = ctrl_mask ? ctrl_mask[g] : 0;
        for (int t = 0; t < k[g]; ++t) m |= 1ull << targets[toff[size_t(g)] + size_t(t)];
        gmask[size_t(g)] = m;
    }
    const uint64_t all = n_qubits >= 64 ? ~0ull : ((1ull << n_qubits) - 1);
    const uint64_t far = far_lo >= 64 ? 0 : (all & ~((1ull << far_lo) - 1));
    int first = 0;
    while (first < n_gates) {
        while (first < n_gates && out.block_of_gate[size_t(first)] >= 0) ++first;
        if (first >= n_gates) break;
        const int b = int(out.block_gates.size());
        out.block_gates.emplace_back();
        uint64_t q = gmask[size_t(first)];
        out.block_of_gate[size_t(first)] = b;
        out.block_gates.back().push_back(first);
        if (__builtin_popcountll(q) <= max_k) {
            uint64_t blocked = 0;
            for (int g = first + 1; g < n_gates; ++g) {
                // stop once no gate can join: every free qubit is blocked, or
                // the block is full and all of its own qubits are blocked
                const uint64_t avail = all & ~blocked;
                if (!avail || (!(q & avail) && __builtin_popcountll(q) >= max_k)) break;
                if (out.block_of_gate[size_t(g)] >= 0) continue;
                const uint64_t m = gmask[size_t(g)];
                if (m & blocked) {
                    blocked |= m;
                    continue;
                }
                const uint64_t u = q | m;
                const bool far_ok = __builtin_popcountll(u & far) <= 1 || (u & far) == (q & far);
                if (__builtin_popcountll(u) <= max_k && far_ok) {
                    q = u;
                    out.block_of_gate[size_t(g)] = b;
                    out.block_gates.back().push_back(g);
                } else {
                    blocked |= m;
                }
            }
        }
        std::vector<int> qs;
        for (int i = 0; i < 64; ++i)
            if ((q >> i) & 1) qs.push_back(i);
        out.block_qubits.push_back(qs);
    }
    return QS_OK;
}

double plan_cost(const Plan &p, int far_lo)
{
    static const double w[] = {1.0, 1.05, 1.10, 1.19, 1.30};
    double c = 0;
    for (const auto &q : p.block_qubits) {
        int f = 0;
        for (int x : q) f += x >= far_lo;
        c += f < 5 ? w[f] : w[4] + 0.1 * (f - 4);
    }
    return c;
}

}  // namespace

int plan_fusion(int n_qubits, int n_gates, const int *k, const int *targets,
                const uint64_t *ctrl_mask, int max_k, Plan &out, int far_lo)
{
    if (int rc = plan_greedy(n_qubits, n_gates, k, targets, ctrl_mask, max_k, out, 64)) return rc;
    if (far_lo >= n_qubits - 1) return QS_OK;        // at most one far qubit: the plans agree
    Plan alt;
    if (int rc = plan_greedy(n_qubits, n_gates, k, targets, ctrl_mask, max_k, alt, far_lo)) return rc;
    if (plan_cost(alt, far_lo) < plan_cost(out, far_lo)) out = std::move(alt);
    return QS_OK;
}

}  // namespace qs
