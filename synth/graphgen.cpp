// Synthetic graph inputs on the host: R-MAT edge generation, deduplication,
// vertex relabelling, symmetric CSR assembly and per-edge weights.
//
// Input generation only: nothing here belongs to the embedding method (no
// walks, negative sampling, training or feedback).  Every random number is
// counter based (SplitMix64 of a seeded counter), so the output depends on
// the seed and the sizes alone, never on the number of threads.
#include <omp.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

inline uint64_t splitmix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Word `word` of the random stream of item `item` under `seed`.
inline uint64_t stream_word(uint64_t seed, uint64_t item, uint64_t word)
{
    return splitmix64(splitmix64(seed ^ 0xD1B54A32D192ED03ull) ^ (item * 16 + word));
}

// Stable LSD radix sort of keys[0, n) on bits [0, bits), 8 bits per pass.
// tmp holds n words.  Returns the buffer holding the result (keys or tmp).
uint64_t* radix_sort(uint64_t* keys, uint64_t* tmp, int64_t n, int bits)
{
    const int nt = omp_get_max_threads();
    std::vector<int64_t> hist((size_t)nt * 256);
    uint64_t* src = keys;
    uint64_t* dst = tmp;
    for (int shift = 0; shift < bits; shift += 8) {
        std::fill(hist.begin(), hist.end(), 0);
#pragma omp parallel num_threads(nt)
        {
            const int t = omp_get_thread_num();
            const int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
            int64_t* h = &hist[(size_t)t * 256];
            for (int64_t i = lo; i < hi; ++i) ++h[(src[i] >> shift) & 255];
#pragma omp barrier
#pragma omp single
            {
                int64_t run = 0;
                for (int d = 0; d < 256; ++d)
                    for (int u = 0; u < nt; ++u) {
                        const int64_t c = hist[(size_t)u * 256 + d];
                        hist[(size_t)u * 256 + d] = run;
                        run += c;
                    }
            }
            for (int64_t i = lo; i < hi; ++i) dst[h[(src[i] >> shift) & 255]++] = src[i];
        }
        std::swap(src, dst);
    }
    return src;
}

int bits_of(uint64_t x)
{
    int b = 0;
    while (b < 64 && (x >> b) != 0) ++b;
    return b;
}

// Group m (row, col) items by row: indptr[n_rows + 1] and cols[m] with each
// row's columns sorted ascending.  The placement within a row follows the
// threads' timing, and the sort makes it deterministic.
template <class RowOf, class ColOf>
void group_by_row(int64_t n_rows, int64_t m, RowOf row_of, ColOf col_of, int64_t* indptr,
                  uint32_t* cols)
{
    std::vector<int64_t> cursor((size_t)n_rows + 1, 0);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        const int64_t r = row_of(i);
#pragma omp atomic
        ++cursor[r + 1];
    }
    for (int64_t r = 0; r < n_rows; ++r) cursor[r + 1] += cursor[r];
    std::copy(cursor.begin(), cursor.end(), indptr);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        const int64_t r = row_of(i);
        int64_t at;
#pragma omp atomic capture
        at = cursor[r]++;
        cols[at] = col_of(i);
    }
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t r = 0; r < n_rows; ++r) std::sort(cols + indptr[r], cols + indptr[r + 1]);
}

}  // namespace

extern "C" {

// Weight of undirected edge {u, v} (order irrelevant): uniform on (0, 1] with
// 2^-24 spacing, ((h >> 40) + 1) 2^-24 for h = SplitMix64 of the edge's key.
float gg_edge_weight(int64_t u, int64_t v, uint64_t seed)
{
    const uint64_t a = (uint64_t)std::min(u, v), b = (uint64_t)std::max(u, v);
    const uint64_t h = stream_word(seed, (a << 32) | b, 0);
    return (float)((double)((h >> 40) + 1) * 0x1p-24);
}

// R-MAT: n_edges distinct undirected edges (u < v) on 2^scale nodes.
// Candidate edge i takes `scale` quadrant choices, one per 16-bit draw r
// (word i of its stream, four draws per 64-bit word): quadrant 0 if r < ta,
// 1 (column bit set) if r < tab, 2 (row bit set) if r < tabc, else 3.
// Candidates are made in rounds until the distinct non-loop edges number at
// least n_edges; the surplus is dropped by keeping the n_edges edges with the
// smallest hash.  With `permute`, vertex v becomes perm[v] for a seeded
// random permutation.  Output: u[n_edges], v[n_edges] sorted by (u, v).
// Returns 0, or -1 if the sizes are out of range.
int gg_rmat(int scale, int64_t n_edges, uint32_t ta, uint32_t tab, uint32_t tabc, uint64_t seed,
            int permute, int64_t* out_u, int64_t* out_v)
{
    if (scale < 1 || scale > 30 || n_edges < 0) return -1;
    const uint64_t n = 1ull << scale;
    if ((uint64_t)n_edges > n * (n - 1) / 2) return -1;
    std::vector<uint64_t> keys;     // distinct keys (u << scale) | v, sorted
    int64_t made = 0;               // candidates made so far
    const int words = (scale + 3) / 4;
    const uint64_t loop_mark = ~0ull;
    std::vector<int64_t> indptr((size_t)n + 1);
    std::vector<uint32_t> cols;
    while ((int64_t)keys.size() < n_edges) {
        const int64_t missing = n_edges - (int64_t)keys.size();
        const int64_t batch = (int64_t)(missing * 1.25) + 4096;
        const size_t old = keys.size();
        keys.resize(old + (size_t)batch);
        uint64_t* out = keys.data() + old;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < batch; ++i) {
            const uint64_t id = (uint64_t)(made + i);
            uint64_t src = 0, dst = 0;
            for (int w = 0; w < words; ++w) {
                uint64_t x = stream_word(seed, id, (uint64_t)w);
                for (int k = 0; k < 4 && 4 * w + k < scale; ++k, x >>= 16) {
                    const uint32_t r = (uint32_t)(x & 0xFFFF);
                    const uint32_t q = (r >= ta) + (r >= tab) + (r >= tabc);
                    src = (src << 1) | (q >> 1);
                    dst = (dst << 1) | (q & 1);
                }
            }
            const uint64_t a = std::min(src, dst), b = std::max(src, dst);
            out[i] = a == b ? loop_mark : (a << scale) | b;
        }
        made += batch;
        // drop the self loops, group by row, keep each (row, col) once
        int64_t m0 = 0;
        for (size_t i = 0; i < keys.size(); ++i)
            if (keys[i] != loop_mark) keys[m0++] = keys[i];
        keys.resize((size_t)m0);
        cols.resize((size_t)m0);
        group_by_row((int64_t)n, m0, [&](int64_t i) { return (int64_t)(keys[i] >> scale); },
                     [&](int64_t i) { return (uint32_t)(keys[i] & (n - 1)); }, indptr.data(),
                     cols.data());
        std::vector<int64_t> kept((size_t)n + 1, 0);
#pragma omp parallel for schedule(dynamic, 4096)
        for (int64_t r = 0; r < (int64_t)n; ++r) {
            int64_t k = 0;
            for (int64_t j = indptr[r]; j < indptr[r + 1]; ++j)
                if (j == indptr[r] || cols[j] != cols[j - 1]) ++k;
            kept[r + 1] = k;
        }
        for (int64_t r = 0; r < (int64_t)n; ++r) kept[r + 1] += kept[r];
        keys.resize((size_t)kept[n]);
#pragma omp parallel for schedule(dynamic, 4096)
        for (int64_t r = 0; r < (int64_t)n; ++r) {
            int64_t at = kept[r];
            for (int64_t j = indptr[r]; j < indptr[r + 1]; ++j)
                if (j == indptr[r] || cols[j] != cols[j - 1])
                    keys[at++] = ((uint64_t)r << scale) | cols[j];
        }
    }
    const uint64_t drop_seed = seed ^ 0xA0761D6478BD642Full;
    if ((int64_t)keys.size() > n_edges) {
        std::vector<uint64_t> h(keys.size());
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < (int64_t)keys.size(); ++i) h[i] = stream_word(drop_seed, keys[i], 1);
        std::vector<uint64_t> hs(h);
        std::nth_element(hs.begin(), hs.begin() + (n_edges - 1), hs.end());
        const uint64_t cut = hs[n_edges - 1];   // keep h < cut, then h == cut in key order
        int64_t below = 0;
        for (uint64_t x : h) below += x < cut;
        int64_t m = 0, eq = 0;
        for (size_t i = 0; i < keys.size(); ++i)
            if (h[i] < cut || (h[i] == cut && eq++ < n_edges - below)) keys[m++] = keys[i];
        keys.resize((size_t)m);
    }
    std::vector<uint64_t> perm;
    if (permute) {
        // perm = the order of the nodes by a random 64-bit value
        std::vector<uint64_t> r(n), tmp(n);
        const int ib = bits_of(n - 1);
        const uint64_t perm_seed = seed ^ 0xE7037ED1A0B428DBull;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < (int64_t)n; ++i)
            r[i] = (stream_word(perm_seed, (uint64_t)i, 2) << ib) | (uint64_t)i;
        uint64_t* s = radix_sort(r.data(), tmp.data(), (int64_t)n, 64);
        perm.resize(n);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < (int64_t)n; ++i) perm[i] = s[i] & (n - 1);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < (int64_t)keys.size(); ++i) {
            const uint64_t a = perm[keys[i] >> scale], b = perm[keys[i] & (n - 1)];
            keys[i] = (std::min(a, b) << scale) | std::max(a, b);
        }
        cols.resize(keys.size());
        group_by_row((int64_t)n, (int64_t)keys.size(),
                     [&](int64_t i) { return (int64_t)(keys[i] >> scale); },
                     [&](int64_t i) { return (uint32_t)(keys[i] & (n - 1)); }, indptr.data(),
                     cols.data());
#pragma omp parallel for schedule(dynamic, 4096)
        for (int64_t r = 0; r < (int64_t)n; ++r)
            for (int64_t j = indptr[r]; j < indptr[r + 1]; ++j)
                keys[j] = ((uint64_t)r << scale) | cols[j];
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)keys.size(); ++i) {
        out_u[i] = (int64_t)(keys[i] >> scale);
        out_v[i] = (int64_t)(keys[i] & (n - 1));
    }
    return 0;
}

// Symmetric CSR from m distinct undirected edges (u[i] != v[i], both in
// [0, n)): indptr[n + 1], indices[2 m] sorted within each row.  weights
// (nullable): the per-edge hash weight of gg_edge_weight under weight_seed.
// Returns 0, or -1 on an out-of-range id.
int gg_csr(int64_t n, int64_t m, const int64_t* u, const int64_t* v, int64_t* indptr,
           int32_t* indices, float* weights, uint64_t weight_seed)
{
    if (n <= 0 || n > ((int64_t)1 << 31)) return -1;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t i = 0; i < m; ++i)
        if (u[i] < 0 || u[i] >= n || v[i] < 0 || v[i] >= n || u[i] == v[i]) bad |= 1;
    if (bad) return -1;
    group_by_row(n, 2 * m, [&](int64_t i) { return i < m ? u[i] : v[i - m]; },
                 [&](int64_t i) { return (uint32_t)(i < m ? v[i] : u[i - m]); }, indptr,
                 reinterpret_cast<uint32_t*>(indices));
    if (weights) {
#pragma omp parallel for schedule(dynamic, 4096)
        for (int64_t r = 0; r < n; ++r)
            for (int64_t j = indptr[r]; j < indptr[r + 1]; ++j)
                weights[j] = gg_edge_weight(r, indices[j], weight_seed);
    }
    return 0;
}

}  // extern "C"

// Indices of k items of [0, m) drawn without replacement (the k smallest
// hashes under `seed`, ties by index), ascending.
static void pick_k(int64_t m, int64_t k, uint64_t seed, uint64_t word, const uint64_t* ids,
                   std::vector<int64_t>& out)
{
    out.clear();
    if (k <= 0) return;
    std::vector<uint64_t> h((size_t)m);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) h[i] = stream_word(seed, ids ? ids[i] : (uint64_t)i, word);
    std::vector<uint64_t> hs(h);
    std::nth_element(hs.begin(), hs.begin() + (k - 1), hs.end());
    const uint64_t cut = hs[k - 1];
    int64_t below = 0;
    for (uint64_t x : h) below += x < cut;
    int64_t eq = 0;
    for (int64_t i = 0; i < m; ++i)
        if (h[i] < cut || (h[i] == cut && eq++ < k - below)) out.push_back(i);
}

extern "C" {

// Link-prediction split of m distinct undirected edges (u < v): n_test of
// them held out (test_idx, ascending), and n_test node pairs u < v that are
// not edges, distinct (neg_u, neg_v, sorted by (u, v)).  Returns 0, or -1 if
// there are not enough non-edges.
int gg_holdout(int64_t n, int64_t m, const int64_t* u, const int64_t* v, int64_t n_test,
               uint64_t seed, int64_t* test_idx, int64_t* neg_u, int64_t* neg_v)
{
    if (n_test < 0 || n_test > m || n < 2) return -1;
    if ((uint64_t)n_test + (uint64_t)m > (uint64_t)n * (uint64_t)(n - 1) / 2) return -1;
    std::vector<int64_t> pick;
    pick_k(m, n_test, seed ^ 0x8BB84B93962EACC9ull, 3, nullptr, pick);
    std::copy(pick.begin(), pick.end(), test_idx);
    // the full edge set, sorted, for membership
    std::vector<uint64_t> full((size_t)m), tmp((size_t)m);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) full[i] = (uint64_t)u[i] * (uint64_t)n + (uint64_t)v[i];
    if (!std::is_sorted(full.begin(), full.end())) {
        uint64_t* s = radix_sort(full.data(), tmp.data(), m, bits_of((uint64_t)n * n - 1));
        if (s != full.data()) std::memcpy(full.data(), s, sizeof(uint64_t) * m);
    }
    const uint64_t neg_seed = seed ^ 0x4F1BBCDCBFA54B11ull;
    std::vector<uint64_t> cand;   // distinct non-edges, sorted
    int64_t made = 0;
    while ((int64_t)cand.size() < n_test) {
        const int64_t batch = 2 * (n_test - (int64_t)cand.size()) + 64;
        std::vector<uint64_t> c((size_t)batch);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < batch; ++i) {
            const uint64_t x = stream_word(neg_seed, (uint64_t)(made + i), 4);
            const uint64_t a = ((x >> 32) * (uint64_t)n) >> 32;
            const uint64_t b = ((x & 0xFFFFFFFFull) * (uint64_t)n) >> 32;
            const uint64_t lo = std::min(a, b), hi = std::max(a, b);
            const uint64_t key = lo * (uint64_t)n + hi;
            const bool edge = std::binary_search(full.begin(), full.end(), key);
            c[i] = (lo == hi || edge) ? ~0ull : key;
        }
        made += batch;
        c.insert(c.end(), cand.begin(), cand.end());
        std::vector<uint64_t> t2(c.size());
        uint64_t* s = radix_sort(c.data(), t2.data(), (int64_t)c.size(), 64);
        cand.clear();
        for (size_t i = 0; i < c.size(); ++i)
            if (s[i] != ~0ull && (cand.empty() || s[i] != cand.back())) cand.push_back(s[i]);
    }
    pick_k((int64_t)cand.size(), n_test, seed ^ 0x2545F4914F6CDD1Dull, 5, cand.data(), pick);
    for (int64_t i = 0; i < n_test; ++i) {
        neg_u[i] = (int64_t)(cand[pick[i]] / (uint64_t)n);
        neg_v[i] = (int64_t)(cand[pick[i]] % (uint64_t)n);
    }
    return 0;
}

}  // extern "C"
