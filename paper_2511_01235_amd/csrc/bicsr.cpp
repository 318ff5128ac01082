// Host construction of the Bi-CSR residual graph (Section 5.1): every vertex
// row lists all of its neighbours, out- and in-, once each and sorted by
// column; an absent reverse direction is a zero-capacity entry, and every
// entry records the index of its reverse entry.  Rows get free slack at the
// end for pairs inserted by later update batches.
#include <algorithm>
#include <climits>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>

#include "mf_internal.h"

namespace mf {

namespace {

int64_t slack_for(int64_t len, int32_t slack_min, int32_t slack_pct) {
    int64_t s = (len * slack_pct + 99) / 100;
    return s < slack_min ? slack_min : s;
}

// Counting sort of (row, col, value) triples by row, then each row by col.
struct RowSorted {
    std::vector<int64_t> beg;   // n+1
    std::vector<int32_t> col;
    std::vector<int64_t> val;
};

void sort_by_row_then_col(int32_t n, int64_t count, const int32_t* row, const int32_t* col,
                          const int64_t* val, RowSorted* out) {
    out->beg.assign((size_t)n + 1, 0);
    for (int64_t i = 0; i < count; ++i) out->beg[(size_t)row[i] + 1]++;
    for (int32_t v = 0; v < n; ++v) out->beg[(size_t)v + 1] += out->beg[(size_t)v];
    std::vector<int64_t> fill(out->beg.begin(), out->beg.end() - 1);
    std::vector<std::pair<int32_t, int64_t>> tmp((size_t)count);
    for (int64_t i = 0; i < count; ++i) tmp[(size_t)fill[(size_t)row[i]]++] = {col[i], val[i]};
    for (int32_t v = 0; v < n; ++v)
        std::sort(tmp.begin() + out->beg[(size_t)v], tmp.begin() + out->beg[(size_t)v + 1],
                  [](const std::pair<int32_t, int64_t>& a, const std::pair<int32_t, int64_t>& b) {
                      return a.first < b.first;
                  });
    out->col.resize((size_t)count);
    out->val.resize((size_t)count);
    for (int64_t i = 0; i < count; ++i) {
        out->col[(size_t)i] = tmp[(size_t)i].first;
        out->val[(size_t)i] = tmp[(size_t)i].second;
    }
}

// Pair every slot with its reverse.  Rows are sorted by column and every
// adjacency is present in both rows, so walking rows in increasing order
// meets the reverse slots of row v in v's own order: a cursor per row gives
// each reverse position in O(1).
void link_reverse(int32_t n, const std::vector<int32_t>& row_ptr, const std::vector<int32_t>& row_len,
                  const std::vector<int32_t>& col, std::vector<int32_t>* rev) {
    std::vector<int32_t> cursor((size_t)n, 0);
    for (int32_t u = 0; u < n; ++u)
        for (int32_t k = 0; k < row_len[(size_t)u]; ++k) {
            int32_t j = row_ptr[(size_t)u] + k;
            int32_t v = col[(size_t)j];
            (*rev)[(size_t)j] = row_ptr[(size_t)v] + cursor[(size_t)v]++;
        }
}

}  // namespace

mf_status build_bicsr(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                      const int32_t* cap, int32_t s, int32_t t, int32_t slack_min,
                      int32_t slack_pct, HostBiCSR* out) {
    if (n < 2 || m < 0 || s < 0 || s >= n || t < 0 || t >= n || s == t) return MF_ERR_INVALID;
    if (m > 0 && (!src || !dst || !cap)) return MF_ERR_INVALID;
    for (int64_t i = 0; i < m; ++i) {
        int32_t u = src[i], v = dst[i];
        if (u < 0 || u >= n || v < 0 || v >= n || u == v || cap[i] < 0) return MF_ERR_INVALID;
    }
    // 1. merge repeated (u,v): sort by row then column, sum runs
    std::vector<int64_t> capv((size_t)m);
    for (int64_t i = 0; i < m; ++i) capv[(size_t)i] = cap[i];
    RowSorted raw;
    sort_by_row_then_col(n, m, src, dst, capv.data(), &raw);
    std::vector<int32_t> pu, pv;
    std::vector<int64_t> pc;
    pu.reserve((size_t)m);
    pv.reserve((size_t)m);
    pc.reserve((size_t)m);
    for (int32_t u = 0; u < n; ++u)
        for (int64_t k = raw.beg[(size_t)u]; k < raw.beg[(size_t)u + 1]; ++k) {
            if (!pu.empty() && pu.back() == u && pv.back() == raw.col[(size_t)k])
                pc.back() += raw.val[(size_t)k];
            else {
                pu.push_back(u);
                pv.push_back(raw.col[(size_t)k]);
                pc.push_back(raw.val[(size_t)k]);
            }
        }
    raw = RowSorted();
    int64_t np = (int64_t)pu.size();
    for (int64_t i = 0; i < np; ++i)
        if (pc[(size_t)i] > INT_MAX) return MF_ERR_OVERFLOW;
    // 2. one entry per direction of every adjacent unordered pair: (u,v,c) in
    //    row u, and a zero-capacity (v,u,0) in row v, merged where both exist
    std::vector<int32_t> er((size_t)(2 * np)), ec((size_t)(2 * np));
    std::vector<int64_t> ev((size_t)(2 * np));
    for (int64_t i = 0; i < np; ++i) {
        er[(size_t)(2 * i)] = pu[(size_t)i];
        ec[(size_t)(2 * i)] = pv[(size_t)i];
        ev[(size_t)(2 * i)] = pc[(size_t)i];
        er[(size_t)(2 * i + 1)] = pv[(size_t)i];
        ec[(size_t)(2 * i + 1)] = pu[(size_t)i];
        ev[(size_t)(2 * i + 1)] = 0;
    }
    RowSorted bi;
    sort_by_row_then_col(n, 2 * np, er.data(), ec.data(), ev.data(), &bi);
    er.clear(); er.shrink_to_fit();
    ec.clear(); ec.shrink_to_fit();
    ev.clear(); ev.shrink_to_fit();
    // merge the (at most two) entries per (row, col)
    std::vector<int32_t> len((size_t)n, 0);
    std::vector<int32_t> col;
    std::vector<int64_t> cval;
    col.reserve((size_t)(2 * np));
    cval.reserve((size_t)(2 * np));
    for (int32_t u = 0; u < n; ++u)
        for (int64_t k = bi.beg[(size_t)u]; k < bi.beg[(size_t)u + 1]; ++k) {
            if (len[(size_t)u] > 0 && col.back() == bi.col[(size_t)k])
                cval.back() += bi.val[(size_t)k];
            else {
                col.push_back(bi.col[(size_t)k]);
                cval.push_back(bi.val[(size_t)k]);
                len[(size_t)u]++;
            }
        }
    bi = RowSorted();
    // 3. rows with slack
    int64_t total = 0;
    out->n = n;
    out->row_ptr.assign((size_t)n + 1, 0);
    for (int32_t v = 0; v < n; ++v) {
        if (total > INT_MAX) return MF_ERR_OVERFLOW;
        out->row_ptr[(size_t)v] = (int32_t)total;
        total += len[(size_t)v] + slack_for(len[(size_t)v], slack_min, slack_pct);
    }
    if (total > INT_MAX) return MF_ERR_OVERFLOW;
    out->row_ptr[(size_t)n] = (int32_t)total;
    out->row_len = len;
    out->row_sorted = len;
    out->col.assign((size_t)total, 0);
    out->cap.assign((size_t)total, 0);
    out->rev.assign((size_t)total, -1);
    int64_t k = 0;
    out->m_unique = 0;
    for (int32_t v = 0; v < n; ++v) {
        int32_t base = out->row_ptr[(size_t)v];
        for (int32_t q = 0; q < len[(size_t)v]; ++q, ++k) {
            out->col[(size_t)(base + q)] = col[(size_t)k];
            out->cap[(size_t)(base + q)] = (int32_t)cval[(size_t)k];
            if (cval[(size_t)k] > 0) out->m_unique++;
        }
        // slack slots point at their own row so that no index can leave [0, n)
        for (int32_t q = len[(size_t)v]; q < out->row_ptr[(size_t)v + 1] - base; ++q)
            out->col[(size_t)(base + q)] = v;
    }
    link_reverse(n, out->row_ptr, out->row_len, out->col, &out->rev);
    // 4. pair sums must fit: res(u,v) + res(v,u) = c(u,v) + c(v,u)
    for (int32_t u = 0; u < n; ++u)
        for (int32_t q = 0; q < len[(size_t)u]; ++q) {
            int32_t j = out->row_ptr[(size_t)u] + q;
            if ((int64_t)out->cap[(size_t)j] + out->cap[(size_t)out->rev[(size_t)j]] > INT_MAX)
                return MF_ERR_OVERFLOW;
        }
    out->pairs = (int64_t)col.size();
    return MF_OK;
}

}  // namespace mf
