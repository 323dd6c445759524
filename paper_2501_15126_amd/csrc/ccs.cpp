// ccs.cpp -- input validation, normalisation and the structural check.
//
// The CCS (compressed sparse column) layout is the paper's CSC of Sec. II:
// cptrs/rids/cvals, here colptr/rowidx/val.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <queue>

#include "perm_internal.h"

namespace permx {

perm_status normalize_ccs(const perm_csc *a, Ccs *out, std::string *err) {
    char buf[256];
    if (!a) {
        *err = "null matrix";
        return PERM_EINVAL;
    }
    const int n = a->n;
    if (n < 1) {
        *err = "n must be >= 1";
        return PERM_EINVAL;
    }
    if (n > PERM_MAX_N) {
        snprintf(buf, sizeof buf, "n = %d exceeds PERM_MAX_N = %d", n, PERM_MAX_N);
        *err = buf;
        return PERM_ETOOBIG;
    }
    if (!a->colptr) {
        *err = "null colptr";
        return PERM_EINVAL;
    }
    if (a->colptr[0] != 0) {
        *err = "colptr[0] must be 0";
        return PERM_EINVAL;
    }
    for (int j = 0; j < n; ++j) {
        if (a->colptr[j + 1] < a->colptr[j]) {
            snprintf(buf, sizeof buf, "colptr decreases at column %d", j);
            *err = buf;
            return PERM_EINVAL;
        }
    }
    const int64_t nnz = a->colptr[n];
    if (nnz > (int64_t)n * n) {
        *err = "more stored entries than n*n";
        return PERM_EINVAL;
    }
    if (nnz > 0 && (!a->rowidx || !a->val)) {
        *err = "null rowidx or val";
        return PERM_EINVAL;
    }
    out->n = n;
    out->colptr.assign(n + 1, 0);
    out->rowidx.clear();
    out->val.clear();
    out->rowidx.reserve(nnz);
    out->val.reserve(nnz);
    for (int j = 0; j < n; ++j) {
        int prev = -1;
        for (int p = a->colptr[j]; p < a->colptr[j + 1]; ++p) {
            const int r = a->rowidx[p];
            const double v = a->val[p];
            if (r < 0 || r >= n) {
                snprintf(buf, sizeof buf, "row index %d out of range in column %d", r, j);
                *err = buf;
                return PERM_EINVAL;
            }
            if (r <= prev) {
                snprintf(buf, sizeof buf, "row indices not strictly increasing in column %d", j);
                *err = buf;
                return PERM_EINVAL;
            }
            if (!std::isfinite(v)) {
                snprintf(buf, sizeof buf, "non-finite value at row %d column %d", r, j);
                *err = buf;
                return PERM_EINVAL;
            }
            prev = r;
            if (v == 0.0) continue;  // explicit zero: not a structural entry
            out->rowidx.push_back(r);
            out->val.push_back(v);
        }
        out->colptr[j + 1] = (int32_t)out->rowidx.size();
    }
    return PERM_OK;
}

// Hopcroft-Karp maximum matching on the bipartite (column, row) graph.
int structural_rank(const Ccs &a) {
    const int n = a.n;
    const int INF = 1 << 30;
    std::vector<int> match_col(n, -1), match_row(n, -1), dist(n);
    auto bfs = [&]() {
        std::queue<int> q;
        bool found = false;
        for (int j = 0; j < n; ++j) {
            if (match_col[j] < 0) {
                dist[j] = 0;
                q.push(j);
            } else {
                dist[j] = INF;
            }
        }
        while (!q.empty()) {
            int j = q.front();
            q.pop();
            for (int p = a.colptr[j]; p < a.colptr[j + 1]; ++p) {
                int r = a.rowidx[p];
                int j2 = match_row[r];
                if (j2 < 0) {
                    found = true;
                } else if (dist[j2] == INF) {
                    dist[j2] = dist[j] + 1;
                    q.push(j2);
                }
            }
        }
        return found;
    };
    std::vector<int> it(n);
    // iterative DFS along the BFS layers
    auto dfs = [&](int root) {
        std::vector<int> stack{root};
        std::vector<int> via;  // row used to reach stack[i+1] from stack[i]
        while (!stack.empty()) {
            int j = stack.back();
            bool advanced = false;
            for (; it[j] < a.colptr[j + 1] - a.colptr[j]; ++it[j]) {
                int r = a.rowidx[a.colptr[j] + it[j]];
                int j2 = match_row[r];
                if (j2 < 0) {
                    // augment along the path
                    via.push_back(r);
                    for (size_t i = 0; i < stack.size(); ++i) {
                        match_col[stack[i]] = via[i];
                        match_row[via[i]] = stack[i];
                    }
                    return true;
                }
                if (dist[j2] == dist[j] + 1) {
                    via.push_back(r);
                    stack.push_back(j2);
                    ++it[j];
                    advanced = true;
                    break;
                }
            }
            if (!advanced) {
                dist[j] = INF;
                stack.pop_back();
                if (!via.empty()) via.pop_back();
            }
        }
        return false;
    };
    int size = 0;
    while (bfs()) {
        for (int j = 0; j < n; ++j) it[j] = 0;
        for (int j = 0; j < n; ++j)
            if (match_col[j] < 0 && dfs(j)) ++size;
    }
    return size;
}

Ccs permute(const Ccs &a, const std::vector<int> &rowPerm, const std::vector<int> &colPerm) {
    const int n = a.n;
    std::vector<int> rowPos(n);
    for (int i = 0; i < n; ++i) rowPos[rowPerm[i]] = i;
    Ccs b;
    b.n = n;
    b.colptr.assign(n + 1, 0);
    b.rowidx.reserve(a.nnz());
    b.val.reserve(a.nnz());
    std::vector<std::pair<int, double>> col;
    for (int jn = 0; jn < n; ++jn) {
        const int j = colPerm[jn];
        col.clear();
        for (int p = a.colptr[j]; p < a.colptr[j + 1]; ++p) col.push_back({rowPos[a.rowidx[p]], a.val[p]});
        std::sort(col.begin(), col.end(), [](const std::pair<int, double> &x, const std::pair<int, double> &y) {
            return x.first < y.first;
        });
        for (auto &e : col) {
            b.rowidx.push_back(e.first);
            b.val.push_back(e.second);
        }
        b.colptr[jn + 1] = (int32_t)b.rowidx.size();
    }
    return b;
}

}  // namespace permx
