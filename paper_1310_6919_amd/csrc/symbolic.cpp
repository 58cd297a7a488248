// Host symbolic phase (Section 2.1 and Section 3.1 of the paper); see symbolic.h.
#include "symbolic.h"

#include <algorithm>
#include <functional>
#include <numeric>
#include <queue>
#include <set>

namespace sdpc {

int64_t Symbolic::slot(int i, int j) const {
    if (i < j) std::swap(i, j);
    const int b = col_block[j];
    const int F = bl_first[b], w = bl_first[b + 1] - F;
    const int64_t r0 = bl_rptr[b];
    const int h = int(bl_rptr[b + 1] - r0);
    int p;
    if (i < F + w) {
        p = i - F;
    } else {
        const int *lo = bl_rows.data() + r0 + w, *hi = bl_rows.data() + r0 + h;
        const int *it = std::lower_bound(lo, hi, i);
        if (it == hi || *it != i) return -1;
        p = int(it - (bl_rows.data() + r0));
    }
    return bl_off[b] + p + int64_t(h) * (j - F);
}

std::vector<int> min_degree_order(int n, const std::vector<int> &arow, const std::vector<int> &acol) {
    std::vector<std::set<int>> adj(n);
    for (size_t t = 0; t < arow.size(); ++t)
        if (arow[t] != acol[t]) {
            adj[arow[t]].insert(acol[t]);
            adj[acol[t]].insert(arow[t]);
        }
    // bucket queue keyed by (degree, index)
    std::set<std::pair<int, int>> q;
    for (int v = 0; v < n; ++v) q.insert({int(adj[v].size()), v});
    std::vector<int> order;
    order.reserve(n);
    while (!q.empty()) {
        const int v = q.begin()->second;
        q.erase(q.begin());
        std::vector<int> nb(adj[v].begin(), adj[v].end());
        for (int a : nb) {
            q.erase({int(adj[a].size()), a});
            adj[a].erase(v);
            for (int c : nb)
                if (c != a) adj[a].insert(c);
            q.insert({int(adj[a].size()), a});
        }
        adj[v].clear();
        order.push_back(v);
    }
    return order;
}

namespace {

// Column structures of the Cholesky factor for the pattern in positions.
// lowcols[j] = rows i > j with (i, j) in the pattern.
void symbolic_factor(int n, const std::vector<std::vector<int>> &lowcols, std::vector<int> &parent,
                     std::vector<int64_t> &sptr, std::vector<int> &sidx) {
    parent.assign(n, -1);
    std::vector<std::vector<int>> children(n);
    std::vector<int> mark(n, -1);
    sptr.assign(1, 0);
    sidx.clear();
    std::vector<int> tmp;
    for (int j = 0; j < n; ++j) {
        tmp.clear();
        tmp.push_back(j);
        mark[j] = j;
        for (int i : lowcols[j])
            if (mark[i] != j) { mark[i] = j; tmp.push_back(i); }
        for (int c : children[j])
            for (int64_t t = sptr[c] + 1; t < sptr[c + 1]; ++t) {
                const int i = sidx[t];
                if (i != j && mark[i] != j) { mark[i] = j; tmp.push_back(i); }
            }
        std::sort(tmp.begin(), tmp.end());
        if (tmp.size() > 1) {
            parent[j] = tmp[1];
            children[tmp[1]].push_back(j);
        }
        sidx.insert(sidx.end(), tmp.begin(), tmp.end());
        sptr.push_back(int64_t(sidx.size()));
    }
}

std::vector<std::vector<int>> low_columns(int n, const std::vector<int> &arow, const std::vector<int> &acol,
                                          const std::vector<int> &pos) {
    std::vector<std::vector<int>> low(n);
    for (size_t t = 0; t < arow.size(); ++t) {
        int a = pos[arow[t]], b = pos[acol[t]];
        if (a == b) continue;
        if (a < b) std::swap(a, b);
        low[b].push_back(a);
    }
    return low;
}

}  // namespace

std::string build_symbolic(int n, const std::vector<int> &arow, const std::vector<int> &acol,
                           const SymbolicOptions &opt, Symbolic &S) {
    S = Symbolic();
    S.n = n;
    // ---- ordering
    std::vector<int> order(n);
    if (opt.ordering == 0) {
        std::iota(order.begin(), order.end(), 0);
    } else if (opt.ordering == 1) {
        order = min_degree_order(n, arow, acol);
    } else if (opt.ordering == 2) {
        if (!opt.user_perm) return "ordering 2 needs user_perm";
        std::vector<char> seen(n, 0);
        for (int i = 0; i < n; ++i) {
            const int v = opt.user_perm[i];
            if (v < 0 || v >= n || seen[v]) return "user_perm is not a permutation";
            seen[v] = 1;
            order[i] = v;
        }
    } else {
        return "unknown ordering";
    }
    std::vector<int> pos(n);
    for (int i = 0; i < n; ++i) pos[order[i]] = i;
    // ---- elimination tree for this order, then a stable postorder (children
    //      visited in ascending order), which keeps an order that already is one
    {
        std::vector<int> par;
        std::vector<int64_t> sp;
        std::vector<int> si;
        symbolic_factor(n, low_columns(n, arow, acol, pos), par, sp, si);
        // visit roots and children by the smallest column of their subtree, so
        // that an order which already is a postorder comes out unchanged
        std::vector<int> fd(n);
        for (int j = 0; j < n; ++j) fd[j] = j;
        for (int j = 0; j < n; ++j)
            if (par[j] >= 0) fd[par[j]] = std::min(fd[par[j]], fd[j]);
        std::vector<std::vector<int>> ch(n);
        std::vector<int> roots;
        for (int j = 0; j < n; ++j) (par[j] < 0 ? roots : ch[par[j]]).push_back(j);
        auto by_fd = [&](int a, int b) { return fd[a] < fd[b]; };
        std::sort(roots.begin(), roots.end(), by_fd);
        for (auto &c : ch) std::sort(c.begin(), c.end(), by_fd);
        std::vector<int> post;
        post.reserve(n);
        std::vector<std::pair<int, size_t>> stack;
        for (int r : roots) {
            stack.push_back({r, 0});
            while (!stack.empty()) {
                auto &top = stack.back();
                if (top.second < ch[top.first].size()) {
                    const int c = ch[top.first][top.second++];
                    stack.push_back({c, 0});
                } else {
                    post.push_back(top.first);
                    stack.pop_back();
                }
            }
        }
        std::vector<int> order2(n);
        for (int i = 0; i < n; ++i) order2[i] = order[post[i]];
        order = order2;
        for (int i = 0; i < n; ++i) pos[order[i]] = i;
    }
    S.perm = order;
    S.pos = pos;
    symbolic_factor(n, low_columns(n, arow, acol, pos), S.parent, S.sptr, S.sidx);
    auto slen = [&](int j) { return int(S.sptr[j + 1] - S.sptr[j]); };
    // ---- fundamental supernodes = cliques
    std::vector<int> nchild(n, 0);
    for (int j = 0; j < n; ++j)
        if (S.parent[j] >= 0) nchild[S.parent[j]]++;
    S.cl_first.assign(1, 0);
    for (int j = 0; j + 1 < n; ++j) {
        const bool same = S.parent[j] == j + 1 && nchild[j + 1] == 1 && slen(j) == slen(j + 1) + 1;
        if (!same) S.cl_first.push_back(j + 1);
    }
    if (n > 0) S.cl_first.push_back(n);
    S.ncl = int(S.cl_first.size()) - 1;
    for (int r = 0; r < S.ncl; ++r) S.max_clique = std::max(S.max_clique, slen(S.cl_first[r]));
    // ---- pieces: supernodes cut to at most block_width columns
    const int W = std::max(1, opt.block_width);
    std::vector<std::pair<int, int>> pieces;
    for (int r = 0; r < S.ncl; ++r) {
        int a = S.cl_first[r];
        while (a < S.cl_first[r + 1]) {
            // widest piece whose panel (rows of its first column x width) fits the limit
            const int hrows = slen(a);
            const int wfit = std::min(W, int(opt.max_block_entries / std::max(1, hrows)));
            if (wfit < 1)
                return "column " + std::to_string(a) + " has " + std::to_string(hrows) +
                       " rows, more than one panel holds";
            const int e = std::min(a + wfit, S.cl_first[r + 1]);
            pieces.push_back({a, e});
            a = e;
        }
    }
    // ---- blocks: merge pieces along elimination-tree chains
    S.bl_first.assign(1, 0);
    S.bl_rptr.assign(1, 0);
    S.bl_rows.clear();
    std::vector<int> rows_cur;   // non-own rows of the current block (sorted, > last column)
    auto own_tail = [&](int F, int end, const std::vector<int> &extra) {
        // rows of a block spanning [F, end): structs of its columns beyond end
        std::vector<int> r;
        for (int j = F; j < end; ++j)
            for (int64_t t = S.sptr[j]; t < S.sptr[j + 1]; ++t)
                if (S.sidx[t] >= end) r.push_back(S.sidx[t]);
        r.insert(r.end(), extra.begin(), extra.end());
        std::sort(r.begin(), r.end());
        r.erase(std::unique(r.begin(), r.end()), r.end());
        return r;
    };
    size_t p = 0;
    while (p < pieces.size()) {
        int F = pieces[p].first, end = pieces[p].second;
        std::vector<int> tail = own_tail(F, end, {});
        size_t q = p + 1;
        while (q < pieces.size()) {
            const int a = pieces[q].first, e = pieces[q].second;
            if (a != end || e - F > W) break;
            // a chain (the next piece starts at the parent of the block's last column), or,
            // with merge_siblings, the next subtree in postorder when the tail rows do not
            // grow (the columns share no entries: explicit zeros, E unchanged)
            const bool chain = S.parent[end - 1] == a;
            if (!chain && !opt.merge_siblings) break;
            std::vector<int> t2 = own_tail(F, e, {});
            if (!chain && t2.size() > tail.size()) break;
            if (int64_t(e - F + t2.size()) * (e - F) > opt.max_block_entries) break;
            end = e;
            tail = t2;
            ++q;
        }
        for (int j = F; j < end; ++j) S.bl_rows.push_back(j);
        S.bl_rows.insert(S.bl_rows.end(), tail.begin(), tail.end());
        S.bl_first.push_back(end);
        S.bl_rptr.push_back(int64_t(S.bl_rows.size()));
        p = q;
    }
    S.nb = int(S.bl_first.size()) - 1;
    S.col_block.assign(n, -1);
    S.bl_off.assign(1, 0);
    for (int b = 0; b < S.nb; ++b) {
        const int w = S.bl_first[b + 1] - S.bl_first[b];
        const int h = int(S.bl_rptr[b + 1] - S.bl_rptr[b]);
        if (int64_t(h) * w > opt.max_block_entries)
            return "storage block " + std::to_string(b) + " has " + std::to_string(h) + " x " +
                   std::to_string(w) + " entries, more than the panel limit";
        S.max_h = std::max(S.max_h, h);
        S.max_w = std::max(S.max_w, w);
        for (int j = S.bl_first[b]; j < S.bl_first[b + 1]; ++j) S.col_block[j] = b;
        S.bl_off.push_back(S.bl_off.back() + int64_t(h) * w);
    }
    S.nslot = S.bl_off.back();
    // ---- block tree and subtree ranges (postorder => subtrees are intervals)
    std::vector<int> sub(n, 1);
    for (int j = 0; j < n; ++j)
        if (S.parent[j] >= 0) sub[S.parent[j]] += sub[j];
    S.bl_parent.assign(S.nb, -1);
    S.bl_subfirst.assign(S.nb, 0);
    for (int b = 0; b < S.nb; ++b) {
        const int last = S.bl_first[b + 1] - 1;
        S.bl_parent[b] = S.parent[last] >= 0 ? S.col_block[S.parent[last]] : -1;
        // the block's columns may head several subtrees (merged siblings): the smallest
        // column of their union, an interval in postorder
        int sf = last - sub[last] + 1;
        for (int j = S.bl_first[b]; j < last; ++j) sf = std::min(sf, j - sub[j] + 1);
        S.bl_subfirst[b] = sf;
    }
    // ---- exact-E mask of the storage
    S.isE.assign(size_t(S.nslot), 0);
    for (int j = 0; j < n; ++j)
        for (int64_t t = S.sptr[j]; t < S.sptr[j + 1]; ++t) {
            const int64_t s = S.slot(S.sidx[t], j);
            if (s < 0) return "internal: exact structure entry missing from its block";
            S.isE[size_t(s)] = 1;
        }
    return "";
}

SolveSlots build_solve_slots(const Symbolic &S, bool delay) {
    SolveSlots R;
    const int n = S.n;
    R.fwd.assign(n, -1);
    R.bwd.assign(n, -1);
    // forward: first touch = first block whose non-own rows contain i
    std::vector<int> first_touch(n, -1), last_read(n, -1);
    for (int b = 0; b < S.nb; ++b) {
        const int w = S.bl_first[b + 1] - S.bl_first[b];
        for (int64_t t = S.bl_rptr[b] + w; t < S.bl_rptr[b + 1]; ++t) {
            const int i = S.bl_rows[t];
            if (first_touch[i] < 0) first_touch[i] = b;
            last_read[i] = (last_read[i] < 0) ? b : std::min(last_read[i], b);
        }
    }
    {
        std::vector<std::vector<int>> born(S.nb);
        for (int i = 0; i < n; ++i)
            if (first_touch[i] >= 0) born[first_touch[i]].push_back(i);
        std::priority_queue<int, std::vector<int>, std::greater<int>> freel;
        int used = 0;
        auto release = [&](int b) {
            for (int j = S.bl_first[b]; j < S.bl_first[b + 1]; ++j)
                if (R.fwd[j] >= 0) freel.push(R.fwd[j]);
        };
        for (int b = 0; b < S.nb; ++b) {
            if (!delay) release(b);   // free for the rows born at b
            for (int i : born[b]) {
                int s;
                if (!freel.empty()) { s = freel.top(); freel.pop(); } else { s = used++; }
                R.fwd[i] = s;
            }
            if (delay) release(b);   // free from block b + 1 on
        }
        R.nfwd = used;
        R.birth = first_touch;
    }
    {
        // backward sweep runs b = nb-1 .. 0; row i is born at its own block and
        // dies at the smallest block that reads it
        std::vector<std::vector<int>> dies(S.nb);
        for (int i = 0; i < n; ++i)
            if (last_read[i] >= 0) dies[last_read[i]].push_back(i);
        std::priority_queue<int, std::vector<int>, std::greater<int>> freel;
        int used = 0;
        for (int b = S.nb - 1; b >= 0; --b) {
            if (!delay)
                for (int i : dies[b]) freel.push(R.bwd[i]);   // read at b, then reused by b's rows
            for (int j = S.bl_first[b]; j < S.bl_first[b + 1]; ++j) {
                if (last_read[j] < 0) continue;
                int s;
                if (!freel.empty()) { s = freel.top(); freel.pop(); } else { s = used++; }
                R.bwd[j] = s;
            }
            if (delay)
                for (int i : dies[b]) freel.push(R.bwd[i]);   // read at b, free from b - 1 on
        }
        R.nbwd = used;
    }
    return R;
}

}  // namespace sdpc
