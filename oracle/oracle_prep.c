/* FP64 oracle: preprocessing (test infrastructure only).
 * Greedy vertex coloring (Sec. 3.9), rest-shape data and lumped masses. */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "vbd_oracle.h"
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { int32_t a, b; } Pair;

static int pair_cmp(const void *p, const void *q)
{
    const Pair *x = (const Pair *)p, *y = (const Pair *)q;
    if (x->a != y->a) return x->a < y->a ? -1 : 1;
    if (x->b != y->b) return x->b < y->b ? -1 : 1;
    return 0;
}

/* Sec. 3.9: color vertices so that no force element uses two vertices of the
 * same color.  Adjacency = every pair of distinct vertices sharing a tet or a
 * spring.  First-fit greedy: vertices in ascending id, each takes the smallest
 * color not used by an already colored neighbour. */
int32_t oracle_color_greedy(int32_t n_verts, int32_t n_tets, const int32_t *tets,
                            int32_t n_springs, const int32_t *springs, int32_t *colors)
{
    size_t np = (size_t)n_tets * 12 + (size_t)n_springs * 2;
    Pair *pr = (Pair *)malloc(sizeof(Pair) * (np + 1));
    size_t q = 0;
    for (int t = 0; t < n_tets; ++t)
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b)
                if (a != b) { pr[q].a = tets[4 * t + a]; pr[q].b = tets[4 * t + b]; ++q; }
    for (int s = 0; s < n_springs; ++s) {
        pr[q].a = springs[2 * s]; pr[q].b = springs[2 * s + 1]; ++q;
        pr[q].a = springs[2 * s + 1]; pr[q].b = springs[2 * s]; ++q;
    }
    qsort(pr, q, sizeof(Pair), pair_cmp);
    int32_t *row = (int32_t *)calloc((size_t)n_verts + 1, sizeof(int32_t));
    for (size_t k = 0; k < q; ++k) row[pr[k].a + 1]++;
    for (int i = 0; i < n_verts; ++i) row[i + 1] += row[i];
    int32_t n_colors = 0;
    int32_t *used = (int32_t *)calloc((size_t)n_verts + 2, sizeof(int32_t));
    for (int v = 0; v < n_verts; ++v) {
        /* mark colors of lower-id neighbours with the stamp v+1 */
        for (int k = row[v]; k < row[v + 1]; ++k) {
            int u = pr[k].b;
            if (u < v) used[colors[u]] = v + 1;
        }
        int c = 0;
        while (used[c] == v + 1) ++c;
        colors[v] = c;
        if (c + 1 > n_colors) n_colors = c + 1;
    }
    free(used); free(row); free(pr);
    return n_colors;
}

/* binary min-heap of (degree, vertex) keys, lexicographic */
typedef struct { int64_t *k; size_t n; } Heap;

static int64_t hkey(int32_t deg, int32_t v) { return ((int64_t)deg << 32) | (int64_t)(uint32_t)v; }

static void heap_push(Heap *h, int64_t key)
{
    size_t i = h->n++;
    h->k[i] = key;
    while (i > 0) {
        size_t parent = (i - 1) / 2;
        if (h->k[parent] <= h->k[i]) break;
        int64_t t = h->k[parent]; h->k[parent] = h->k[i]; h->k[i] = t;
        i = parent;
    }
}

static int64_t heap_pop(Heap *h)
{
    int64_t top = h->k[0];
    h->k[0] = h->k[--h->n];
    size_t i = 0;
    for (;;) {
        size_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < h->n && h->k[l] < h->k[m]) m = l;
        if (r < h->n && h->k[r] < h->k[m]) m = r;
        if (m == i) break;
        int64_t t = h->k[m]; h->k[m] = h->k[i]; h->k[i] = t;
        i = m;
    }
    return top;
}

/* Greedy first fit over the smallest-last order (Matula and Beck, J. ACM
 * 30(3), 1983): repeatedly remove a vertex of smallest degree among the
 * remaining ones (ties: smallest id); color in the reverse of the removal
 * order, each vertex taking the smallest color not used by an already
 * colored neighbour.  Same adjacency as oracle_color_greedy. */
int32_t oracle_color_smallest_last(int32_t n_verts, int32_t n_tets, const int32_t *tets,
                                   int32_t n_springs, const int32_t *springs, int32_t *colors)
{
    size_t np = (size_t)n_tets * 12 + (size_t)n_springs * 2;
    Pair *pr = (Pair *)malloc(sizeof(Pair) * (np + 1));
    size_t q = 0;
    for (int t = 0; t < n_tets; ++t)
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b)
                if (a != b) { pr[q].a = tets[4 * t + a]; pr[q].b = tets[4 * t + b]; ++q; }
    for (int s = 0; s < n_springs; ++s) {
        pr[q].a = springs[2 * s]; pr[q].b = springs[2 * s + 1]; ++q;
        pr[q].a = springs[2 * s + 1]; pr[q].b = springs[2 * s]; ++q;
    }
    qsort(pr, q, sizeof(Pair), pair_cmp);
    /* drop repeated pairs (an edge shared by several tets) */
    size_t u = 0;
    for (size_t k = 0; k < q; ++k)
        if (u == 0 || pair_cmp(&pr[u - 1], &pr[k]) != 0) pr[u++] = pr[k];
    q = u;
    int32_t *row = (int32_t *)calloc((size_t)n_verts + 1, sizeof(int32_t));
    for (size_t k = 0; k < q; ++k) row[pr[k].a + 1]++;
    for (int i = 0; i < n_verts; ++i) row[i + 1] += row[i];
    int32_t *deg = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n_verts + 1));
    uint8_t *gone = (uint8_t *)calloc((size_t)n_verts + 1, 1);
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n_verts + 1));
    Heap h = {(int64_t *)malloc(sizeof(int64_t) * (q + (size_t)n_verts + 1)), 0};
    for (int v = 0; v < n_verts; ++v) {
        deg[v] = row[v + 1] - row[v];
        heap_push(&h, hkey(deg[v], v));
    }
    int32_t removed = 0;
    while (h.n > 0) {
        int64_t key = heap_pop(&h);
        int32_t v = (int32_t)(key & 0xffffffff), d = (int32_t)(key >> 32);
        if (gone[v] || d != deg[v]) continue;      /* stale entry */
        gone[v] = 1;
        order[removed++] = v;
        for (int k = row[v]; k < row[v + 1]; ++k) {
            int w = pr[k].b;
            if (!gone[w]) { deg[w]--; heap_push(&h, hkey(deg[w], w)); }
        }
    }
    int32_t n_colors = 0;
    int32_t *used = (int32_t *)calloc((size_t)n_verts + 2, sizeof(int32_t));
    for (int v = 0; v < n_verts; ++v) colors[v] = -1;
    for (int i = n_verts - 1; i >= 0; --i) {
        int v = order[i];
        for (int k = row[v]; k < row[v + 1]; ++k) {
            int w = pr[k].b;
            if (colors[w] >= 0) used[colors[w]] = i + 1;
        }
        int c = 0;
        while (used[c] == i + 1) ++c;
        colors[v] = c;
        if (c + 1 > n_colors) n_colors = c + 1;
    }
    free(used); free(h.k); free(order); free(gone); free(deg); free(row); free(pr);
    return n_colors;
}

/* DSATUR (Brelaz, Comm. ACM 22(4), 1979), one more greedy vertex order for
 * the coloring of Sec. 3.9 (any coloring in which no element joins two
 * vertices of one color serves; the paper names no algorithm): repeatedly
 * color the uncolored vertex with the most distinct colors among its
 * neighbours (ties: larger degree, then smaller id) with the smallest color
 * none of its neighbours has.  Same adjacency as oracle_color_greedy. */
int32_t oracle_color_dsatur(int32_t n_verts, int32_t n_tets, const int32_t *tets,
                            int32_t n_springs, const int32_t *springs, int32_t *colors)
{
    size_t np = (size_t)n_tets * 12 + (size_t)n_springs * 2;
    Pair *pr = (Pair *)malloc(sizeof(Pair) * (np + 1));
    size_t q = 0;
    for (int t = 0; t < n_tets; ++t)
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b)
                if (a != b) { pr[q].a = tets[4 * t + a]; pr[q].b = tets[4 * t + b]; ++q; }
    for (int s = 0; s < n_springs; ++s) {
        pr[q].a = springs[2 * s]; pr[q].b = springs[2 * s + 1]; ++q;
        pr[q].a = springs[2 * s + 1]; pr[q].b = springs[2 * s]; ++q;
    }
    qsort(pr, q, sizeof(Pair), pair_cmp);
    size_t u = 0;
    for (size_t k = 0; k < q; ++k)
        if (u == 0 || pair_cmp(&pr[u - 1], &pr[k]) != 0) pr[u++] = pr[k];
    q = u;
    int32_t *row = (int32_t *)calloc((size_t)n_verts + 1, sizeof(int32_t));
    for (size_t k = 0; k < q; ++k) row[pr[k].a + 1]++;
    for (int i = 0; i < n_verts; ++i) row[i + 1] += row[i];
    /* per vertex: saturation count and a bitset of neighbour colors, grown on demand */
    int32_t *sat = (int32_t *)calloc((size_t)n_verts + 1, sizeof(int32_t));
    int32_t words = 1;
    uint64_t *seen = (uint64_t *)calloc((size_t)n_verts * words + 1, sizeof(uint64_t));
    /* heap key, smaller first: (2047 - sat, maxdeg - deg, id) */
    int32_t maxdeg = 0;
    for (int v = 0; v < n_verts; ++v) if (row[v + 1] - row[v] > maxdeg) maxdeg = row[v + 1] - row[v];
    /* the degree field has 20 bits */
    const int64_t SAT_SHIFT = 52, DEG_SHIFT = 32;
    /* 11 bits of saturation keep the key positive (at most 2047 colors) */
    #define DKEY(v, s) ((((int64_t)(2047 - (s))) << SAT_SHIFT) | (((int64_t)(maxdeg - (row[(v) + 1] - row[(v)]))) << DEG_SHIFT) | (int64_t)(uint32_t)(v))
    Heap h = {(int64_t *)malloc(sizeof(int64_t) * (q + (size_t)n_verts + 1)), 0};
    for (int v = 0; v < n_verts; ++v) { colors[v] = -1; heap_push(&h, DKEY(v, 0)); }
    int32_t n_colors = 0;
    while (h.n > 0) {
        int64_t key = heap_pop(&h);
        int32_t v = (int32_t)(key & 0xffffffff);
        int32_t s = 2047 - (int32_t)(key >> SAT_SHIFT);
        if (colors[v] >= 0 || s != sat[v]) continue;      /* stale */
        int c = 0;
        while (c < 64 * words && (seen[(size_t)v * words + (size_t)(c >> 6)] >> (c & 63) & 1ull)) ++c;
        colors[v] = c;
        if (c + 1 > n_colors) n_colors = c + 1;
        if (c >= 64 * words) {
            /* widen every bitset */
            int32_t nw = words * 2;
            uint64_t *ns = (uint64_t *)calloc((size_t)n_verts * nw + 1, sizeof(uint64_t));
            for (int x = 0; x < n_verts; ++x)
                for (int k = 0; k < words; ++k) ns[(size_t)x * nw + k] = seen[(size_t)x * words + k];
            free(seen); seen = ns; words = nw;
        }
        for (int k = row[v]; k < row[v + 1]; ++k) {
            int w = pr[k].b;
            if (colors[w] >= 0) continue;
            uint64_t *bits = seen + (size_t)w * words;
            if (!(bits[c >> 6] >> (c & 63) & 1ull)) {
                bits[c >> 6] |= 1ull << (c & 63);
                sat[w]++;
                heap_push(&h, DKEY(w, sat[w]));
            }
        }
    }
    #undef DKEY
    free(h.k); free(seen); free(sat); free(row); free(pr);
    return n_colors;
}

/* D_m = [X1-X0, X2-X0, X3-X0]; Dminv by Gauss-Jordan elimination with partial
 * pivoting; V = |det D_m| / 6. */
int32_t oracle_tet_rest(int32_t n_tets, const int32_t *tets, const double *rest,
                        double *Dminv, double *vol)
{
    for (int t = 0; t < n_tets; ++t) {
        double A[3][6];
        const double *X0 = rest + 3 * tets[4 * t];
        for (int c = 0; c < 3; ++c) {
            const double *Xc = rest + 3 * tets[4 * t + c + 1];
            for (int r = 0; r < 3; ++r) A[r][c] = Xc[r] - X0[r];
        }
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) A[r][3 + c] = (r == c) ? 1.0 : 0.0;
        double det = 1.0, scale = 0.0;
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) scale = fmax(scale, fabs(A[r][c]));
        for (int col = 0; col < 3; ++col) {
            int piv = col;
            for (int r = col + 1; r < 3; ++r)
                if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
            if (piv != col) {
                for (int c = 0; c < 6; ++c) { double tmp = A[col][c]; A[col][c] = A[piv][c]; A[piv][c] = tmp; }
                det = -det;
            }
            double p = A[col][col];
            det *= p;
            if (fabs(p) <= 1e-300) return -1 - t;
            for (int c = 0; c < 6; ++c) A[col][c] /= p;
            for (int r = 0; r < 3; ++r) {
                if (r == col) continue;
                double fct = A[r][col];
                for (int c = 0; c < 6; ++c) A[r][c] -= fct * A[col][c];
            }
        }
        if (fabs(det) <= 1e-12 * scale * scale * scale) return -1 - t;
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) Dminv[9 * t + 3 * r + c] = A[r][3 + c];
        vol[t] = fabs(det) / 6.0;
    }
    return 0;
}

void oracle_lumped_mass(int32_t n_verts, int32_t n_tets, const int32_t *tets, const double *vol,
                        double density, double *mass)
{
    memset(mass, 0, sizeof(double) * (size_t)n_verts);
    for (int t = 0; t < n_tets; ++t)
        for (int a = 0; a < 4; ++a) mass[tets[4 * t + a]] += density * vol[t] / 4.0;
}

void oracle_spring_rest(int32_t n_springs, const int32_t *springs, const double *rest, double *L)
{
    for (int s = 0; s < n_springs; ++s) {
        const double *a = rest + 3 * springs[2 * s], *b = rest + 3 * springs[2 * s + 1];
        double d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2];
        L[s] = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    }
}

void oracle_set_threads(int32_t n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

typedef struct { int32_t key[3]; int32_t v[3]; int32_t opp; } Face;

static int face_cmp(const void *p, const void *q)
{
    const Face *a = (const Face *)p, *b = (const Face *)q;
    for (int k = 0; k < 3; ++k)
        if (a->key[k] != b->key[k]) return a->key[k] < b->key[k] ? -1 : 1;
    return 0;
}

/* Faces used by exactly one tet, with the normal (b-a) x (c-a) pointing away
 * from the tet's fourth vertex; ordered by their sorted vertex ids. */
int32_t oracle_surface(int32_t n_tets, const int32_t *tets, const double *rest, int32_t *tris_out)
{
    Face *F = (Face *)malloc(sizeof(Face) * (4 * (size_t)n_tets + 1));
    size_t nf = 0;
    for (int t = 0; t < n_tets; ++t)
        for (int o = 0; o < 4; ++o) {
            Face f;
            int k = 0;
            for (int j = 0; j < 4; ++j)
                if (j != o) f.v[k++] = tets[4 * t + j];
            f.opp = tets[4 * t + o];
            int a = f.v[0], b = f.v[1], c = f.v[2], tmp;
            if (a > b) { tmp = a; a = b; b = tmp; }
            if (b > c) { tmp = b; b = c; c = tmp; }
            if (a > b) { tmp = a; a = b; b = tmp; }
            f.key[0] = a; f.key[1] = b; f.key[2] = c;
            F[nf++] = f;
        }
    qsort(F, nf, sizeof(Face), face_cmp);
    int32_t n_out = 0;
    for (size_t i = 0; i < nf;) {
        size_t j = i + 1;
        while (j < nf && face_cmp(&F[i], &F[j]) == 0) ++j;
        if (j - i == 1) {
            const double *A = rest + 3 * F[i].v[0], *B = rest + 3 * F[i].v[1], *Cc = rest + 3 * F[i].v[2];
            const double *D = rest + 3 * F[i].opp;
            double ab[3], ac[3], ad[3];
            for (int k = 0; k < 3; ++k) { ab[k] = B[k] - A[k]; ac[k] = Cc[k] - A[k]; ad[k] = D[k] - A[k]; }
            double n[3] = {ab[1] * ac[2] - ab[2] * ac[1], ab[2] * ac[0] - ab[0] * ac[2], ab[0] * ac[1] - ab[1] * ac[0]};
            int32_t *o = tris_out + 3 * n_out;
            o[0] = F[i].v[0];
            if (n[0] * ad[0] + n[1] * ad[1] + n[2] * ad[2] > 0.0) { o[1] = F[i].v[2]; o[2] = F[i].v[1]; }
            else { o[1] = F[i].v[1]; o[2] = F[i].v[2]; }
            ++n_out;
        }
        i = j;
    }
    free(F);
    return n_out;
}
