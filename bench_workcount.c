/*
 * Work counting for the benchmark's roofline: the nodes, leaf cells and cluster
 * nodes that the hierarchical evaluation of a query must touch by the rules of
 * its descent, independent of how a GPU schedules it.
 *
 * Per query (section "Acceleration by mesh clustering", Fig. acceleration;
 * supplement "Entry level"): support half-widths r = fl32(sigma_to_r sigma), box
 * [x - r, x + r] and the unrolled cell range it meets, entry level
 * l0 = min(L, smallest l with 2^l >= max(r_x, r_y)), cut threshold
 * t = fl32(fl32(r_x r_y) tau).  The roots are every level-l0 node with a periodic
 * image meeting the cell range (cells when l0 = 0).  A visited node counts one box
 * test: with tau > 0 and e^l <= t it is one cluster node (its two triangles
 * tested) when h lies inside its box, which from level 2 up is that of its own two
 * cluster triangles; otherwise it stops when h lies outside its box, at level 1
 * counts its cells that meet the range, and above visits its children that meet
 * the range -- except that a node of level 3 or more reached from its parent (not
 * a root) whose children are all under the cut takes a second box test, the union
 * of its children's own boxes, and stops when h lies outside it (none of their
 * cluster tests could hit).  The boxes are those of the map's triangles (tau = 0) or of the map's
 * and cluster triangles beneath the node (tau > 0), as the hierarchy stores them
 * in float32.
 *
 * Build: gcc -O2 -shared -fPIC -fopenmp bench_workcount.c -o bench_workcount.so
 */
#include <math.h>
#include <stdint.h>

typedef struct {
    int n, L;
    const float* box;  /* levels 1..L packed, row-major nodes, (min x, min y, max x, max y) */
    const float* own;  /* the same for the node's own cluster triangles (NULL when tau = 0) */
    const float* e;    /* levels 1..L packed, row-major nodes (NULL when tau = 0) */
    long off[32];
} hier_t;

typedef struct {
    float hx, hy, t;
    long clo[2], chi[2];
    int cut;
    uint64_t nodes, cells, clusters;
} walk_t;

static long floor_div(long a, long b) { long q = a / b; return (q * b > a) ? q - 1 : q; }

/* does the node (side s, starting cell `start`) have a periodic image meeting
 * the unrolled cell range [lo, hi] of a torus of n cells */
static int axis_meets(long start, long s, long lo, long hi, long n)
{
    /* the first image ending at or after lo starts at start + p n */
    long p = floor_div(lo - start - s + 1 + n - 1, n);
    return start + p * n <= hi;
}

static int inside_box(const float* b, float x, float y)
{
    return x >= b[0] && y >= b[1] && x <= b[2] && y <= b[3];
}

/* are the four children of node (l, I) all under the cut */
static int children_all_cut(const hier_t* h, const walk_t* w, int l, long I, long J)
{
    const long mc = (long)h->n >> (l - 1);
    int all = 1;
    for (int dj = 0; dj < 2; dj++)
        for (int di = 0; di < 2; di++) all &= h->e[h->off[l - 1] + (2 * J + dj) * mc + 2 * I + di] <= w->t;
    return all;
}

/* does the union of the four children's own boxes hold h */
static int children_own_hold(const hier_t* h, const walk_t* w, int l, long I, long J)
{
    const long mc = (long)h->n >> (l - 1);
    int any = 0;
    for (int dj = 0; dj < 2; dj++)
        for (int di = 0; di < 2; di++)
            any |= inside_box(h->own + 4 * (h->off[l - 1] + (2 * J + dj) * mc + 2 * I + di), w->hx, w->hy);
    return any;
}

static void visit(const hier_t* h, walk_t* w, int l, long I, long J, int root)
{
    const long m = (long)h->n >> l;
    const long k = h->off[l] + J * m + I;
    const float* b = h->box + 4 * k;
    w->nodes++;
    if (w->cut && h->e[k] <= w->t) {
        const float* c = l >= 2 ? h->own + 4 * k : b;
        if (w->hx >= c[0] && w->hy >= c[1] && w->hx <= c[2] && w->hy <= c[3]) w->clusters++;
        return;
    }
    if (!(w->hx >= b[0] && w->hy >= b[1] && w->hx <= b[2] && w->hy <= b[3])) return;
    if (w->cut && !root && l >= 3 && children_all_cut(h, w, l, I, J)) {
        w->nodes++;  /* a second box test: the union of the children's own boxes */
        if (!children_own_hold(h, w, l, I, J)) return;
    }
    const long s = 1L << (l - 1);
    for (int dj = 0; dj < 2; dj++)
        for (int di = 0; di < 2; di++) {
            const long ci = 2 * I + di, cj = 2 * J + dj;
            if (!axis_meets(ci * s, s, w->clo[0], w->chi[0], h->n) || !axis_meets(cj * s, s, w->clo[1], w->chi[1], h->n))
                continue;
            if (l == 1)
                w->cells++;
            else
                visit(h, w, l - 1, ci, cj, 0);
        }
}

/*
 * q: nq queries (x, y, sx, sy, hx, hy); out: nq x 3 (nodes, cells, clusters).
 * Invalid queries (as the evaluation defines them) count nothing.
 */
int wc_count(int n, const float* box, const float* own, const float* e, const float* q, int64_t nq, float tau, float s2r,
             uint64_t* out)
{
    hier_t h;
    h.n = n;
    h.L = 0;
    while ((1 << h.L) < n) h.L++;
    if ((1 << h.L) != n || h.L < 1 || h.L > 30) return 1;
    if (tau > 0.0f && (!e || !own)) return 2;
    h.box = box;
    h.own = own;
    h.e = e;
    long off = 0;
    for (int l = 1; l <= h.L; l++) {
        h.off[l] = off;
        off += (long)(n >> l) * (n >> l);
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < nq; k++) {
        const float* r = q + 6 * k;
        walk_t w;
        w.nodes = w.cells = w.clusters = 0;
        const float lim = 16777216.0f;
        const int ok = isfinite(r[0]) && isfinite(r[1]) && isfinite(r[2]) && isfinite(r[3]) && isfinite(r[4]) &&
                       isfinite(r[5]) && r[2] > 0.0f && r[3] > 0.0f;
        const float rx = s2r * r[2], ry = s2r * r[3];
        if (ok && fabsf(r[0]) <= lim && fabsf(r[1]) <= lim && rx <= lim && ry <= lim) {
            const float lox = r[0] - rx, hix = r[0] + rx, loy = r[1] - ry, hiy = r[1] + ry;
            w.clo[0] = (long)ceilf(lox) - 1;
            w.chi[0] = (long)floorf(hix);
            w.clo[1] = (long)ceilf(loy) - 1;
            w.chi[1] = (long)floorf(hiy);
            w.hx = r[4];
            w.hy = r[5];
            const float rr = rx * ry;
            w.t = rr * tau;
            w.cut = tau > 0.0f;
            const float rmax = rx > ry ? rx : ry;
            int l0 = 0;
            while (l0 < h.L && (float)(1L << l0) < rmax) l0++;
            /* the level-l0 columns meeting the range form one cyclic run per axis */
            const long m = (long)n >> l0, s = 1L << l0;
            long a[2], len[2];
            for (int ax = 0; ax < 2; ax++) {
                a[ax] = floor_div(w.clo[ax], s);
                len[ax] = floor_div(w.chi[ax], s) - a[ax] + 1;
                if (len[ax] > m) len[ax] = m;
            }
            for (long y = 0; y < len[1]; y++) {
                const long J = ((a[1] + y) % m + m) % m;
                for (long x = 0; x < len[0]; x++) {
                    const long I = ((a[0] + x) % m + m) % m;
                    if (l0 == 0)
                        w.cells++;
                    else
                        visit(&h, &w, l0, I, J, 1);
                }
            }
        }
        out[3 * k] = w.nodes;
        out[3 * k + 1] = w.cells;
        out[3 * k + 2] = w.clusters;
    }
    return 0;
}
