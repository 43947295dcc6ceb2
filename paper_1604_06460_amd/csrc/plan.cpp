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
#include <algorithm>
#include <cstdint>
#include <vector>

#include "qs_internal.h"

namespace qs {

int plan_fusion(int n_qubits, int n_gates, const int *k, const int *targets,
                const uint64_t *ctrl_mask, int max_k, Plan &out)
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
                if (__builtin_popcountll(q | m) <= max_k) {
                    q |= m;
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

}  // namespace qs
