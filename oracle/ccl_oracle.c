/*
 * CPU oracle for two-pass connected component labeling (Gupta, Palsetia,
 * Patwary, Agrawal, Choudhary, "A New Parallel Algorithm for Two-Pass
 * Connected Component Labeling", arXiv 1606.05973).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this file.  It shares no code with
 * the GPU library and must never be used as a fallback for it.
 *
 * Plain, slow, single-threaded C.  Every routine follows the paper's
 * definitions in the paper's order and notation:
 *   merge        -- Rem's union with splicing (Section III, Algorithm 2)
 *   flatten      -- analysis phase (Section III, Algorithm 3)
 *   cclremsp     -- CCLRemSP: decision-tree scan (Fig. 2, Algorithm 4),
 *                   flatten, labeling phase (Algorithm 1)
 *   aremsp       -- ARemSP: two-row scan with the mask of Fig. 1b
 *                   (Algorithm 6), flatten, labeling (Algorithm 5)
 *   paremsp      -- PARemSP: chunked ARemSP scans with disjoint label
 *                   ranges, boundary-row merge with merger (Algorithms 7, 8)
 *                   executed one chunk after another, flatten, labeling
 *   gray         -- the gray-level extension the paper mentions (Section V;
 *                   the abstract's "adjacent pixels sharing the same
 *                   features"): object pixels are the nonzero bytes and two
 *                   neighbouring object pixels are connected when their
 *                   bytes are equal; same raster scan with merge, flatten,
 *                   labeling
 *   canonical    -- renumbers a labeling so that component k is the k-th
 *                   component met in raster order (the required output
 *                   numbering; not in the paper)
 *
 * Conventions (the readings where the paper is silent or garbled):
 *   - a pixel is foreground when its byte is nonzero (Section III uses 1);
 *   - pixels outside the image are background;
 *   - label 0 is background and p[0] = 0, so the labeling phase may map
 *     every pixel through p; provisional labels start at 1;
 *   - flatten runs over labels 1..(largest label handed out);
 *   - Algorithm 6, case e=1, d=0, b=0, f=1, a=1: the merge is between the
 *     labels of e and a (one argument is missing in the listing);
 *   - Algorithm 6, case e=0, g=1, d=0, f=0: the new label goes to g
 *     (e is background);
 *   - Algorithm 7: chunk k's labels start at start_row*W + 1 so that no
 *     chunk hands out label 0; each chunk's first row is merged against
 *     the previous chunk's last row; the last chunk takes the remainder;
 *   - Algorithm 8: the rootness recheck of the y side tests root_y;
 *   - 4-connectivity is not spelled out in the paper; it is derived from
 *     the same masks with the diagonal neighbours removed.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    const uint8_t *img;
    int64_t H, W, stride;
} image_t;

/* image(x) of Section III: 1 for an object pixel, 0 otherwise. */
static int image_at(const image_t *im, int64_t r, int64_t c)
{
    if (r < 0 || r >= im->H || c < 0 || c >= im->W)
        return 0;
    return im->img[r * im->stride + c] != 0;
}

/* label(x) for a pixel of the provisional label array; 0 outside. */
static int32_t label_at(const int32_t *label, const image_t *im, int64_t r, int64_t c)
{
    if (r < 0 || r >= im->H || c < 0 || c >= im->W)
        return 0;
    return label[r * im->W + c];
}

/* ---------------------------------------------------------------------- */
/* Algorithm 2: merge(p, x, y).  Rem's algorithm with splicing.  The root   */
/* with the larger parent value is linked below the smaller parent value;   */
/* on the way up, the node with the larger parent is spliced onto the other */
/* side's parent.  The invariant p[i] <= i is kept, so every set's root is  */
/* its smallest element.  Returns a member of the united set.               */
/* ---------------------------------------------------------------------- */
static int32_t merge(int32_t *p, int32_t x, int32_t y)
{
    int32_t root_x = x, root_y = y, z;
    while (p[root_x] != p[root_y]) {
        if (p[root_x] > p[root_y]) {
            if (root_x == p[root_x]) {
                p[root_x] = p[root_y];
                return p[root_x];
            }
            z = p[root_x];
            p[root_x] = p[root_y];
            root_x = z;
        } else {
            if (root_y == p[root_y]) {
                p[root_y] = p[root_x];
                return p[root_x];
            }
            z = p[root_y];
            p[root_y] = p[root_x];
            root_y = z;
        }
    }
    return p[root_x];
}

/* Algorithm 8: merger(p, x, y).  The concurrent form of Algorithm 2: a root */
/* is linked only after re-checking, under the lock of that root, that it   */
/* is still a root; splicing is done without locks.  Here the chunks are   */
/* merged one after another, which is one of the schedules the concurrent   */
/* algorithm admits, so the lock reduces to the re-check itself.            */
static int32_t merger(int32_t *p, int32_t x, int32_t y)
{
    int32_t root_x = x, root_y = y, z;
    while (p[root_x] != p[root_y]) {
        if (p[root_x] > p[root_y]) {
            if (root_x == p[root_x]) {
                int success = 0;
                /* lock(root_x) */
                if (root_x == p[root_x]) {
                    p[root_x] = p[root_y];
                    success = 1;
                }
                /* unlock(root_x) */
                if (success)
                    break;
            }
            z = p[root_x];
            p[root_x] = p[root_y];
            root_x = z;
        } else {
            if (root_y == p[root_y]) {
                int success = 0;
                if (root_y == p[root_y]) {
                    p[root_y] = p[root_x];
                    success = 1;
                }
                if (success)
                    break;
            }
            z = p[root_y];
            p[root_y] = p[root_x];
            root_y = z;
        }
    }
    return p[root_x];
}

/* Algorithm 3: flatten(p, count).  One ascending sweep: a non-root takes   */
/* its parent's (already final) value, a root takes the next consecutive    */
/* label.  Returns the number of roots, i.e. of components.                 */
static int32_t flatten(int32_t *p, int32_t count)
{
    int32_t k = 1;
    for (int32_t i = 1; i <= count; i++) {
        if (p[i] < i)
            p[i] = p[p[i]];
        else {
            p[i] = k;
            k++;
        }
    }
    return k - 1;
}

/* Labeling phase (Algorithms 1, 5, 7): label(e) <- p[label(e)] everywhere. */
static void labeling_phase(int32_t *label, const image_t *im, const int32_t *p)
{
    for (int64_t r = 0; r < im->H; r++)
        for (int64_t c = 0; c < im->W; c++)
            label[r * im->W + c] = p[label[r * im->W + c]];
}

/* Upper bound on the number of provisional labels any scan can hand out:   */
/* a new label lands on a foreground pixel whose already-scanned 4-neighbours */
/* are background, so no two new labels sit on 4-adjacent pixels and there  */
/* are at most ceil(H*W/2) of them.                                         */
static int64_t max_labels(int64_t H, int64_t W)
{
    return (H * W + 1) / 2 + 2;
}

/* ---------------------------------------------------------------------- */
/* CCLRemSP scan (Algorithm 4 with the decision tree of Fig. 2).           */
/* Mask of Fig. 1a: a=(r-1,c-1) b=(r-1,c) c=(r-1,c+1) d=(r,c-1), e=(r,c).   */
/* copy(x)   : label(e) = p[label(x)]                                       */
/* copy(x,y) : label(e) = merge(p, label(x), label(y))                      */
/* new label : label(e) = count; p[count] = count; count++                  */
/* Returns the largest label handed out.                                    */
/* ---------------------------------------------------------------------- */
static int32_t scan_cclremsp(const image_t *im, int conn, int32_t *label, int32_t *p)
{
    int32_t count = 1;
    p[0] = 0;
    for (int64_t r = 0; r < im->H; r++) {
        for (int64_t c = 0; c < im->W; c++) {
            int32_t *e = &label[r * im->W + c];
            *e = 0;
            if (!image_at(im, r, c))
                continue;
            int a = image_at(im, r - 1, c - 1), b = image_at(im, r - 1, c);
            int cc = image_at(im, r - 1, c + 1), d = image_at(im, r, c - 1);
            int32_t la = label_at(label, im, r - 1, c - 1), lb = label_at(label, im, r - 1, c);
            int32_t lc = label_at(label, im, r - 1, c + 1), ld = label_at(label, im, r, c - 1);
            if (conn == 8) {
                if (b)
                    *e = p[lb];                       /* copy(b)   */
                else if (cc) {
                    if (a)
                        *e = merge(p, lc, la);        /* copy(c,a) */
                    else if (d)
                        *e = merge(p, lc, ld);        /* copy(c,d) */
                    else
                        *e = p[lc];                   /* copy(c)   */
                } else if (a)
                    *e = p[la];                       /* copy(a)   */
                else if (d)
                    *e = p[ld];                       /* copy(d)   */
                else {
                    *e = count;                       /* new label */
                    p[count] = count;
                    count++;
                }
            } else {
                /* 4-connectivity: only b (above) and d (left) are neighbours. */
                if (b && d)
                    *e = merge(p, lb, ld);
                else if (b)
                    *e = p[lb];
                else if (d)
                    *e = p[ld];
                else {
                    *e = count;
                    p[count] = count;
                    count++;
                }
            }
        }
    }
    return count - 1;
}

/* ---------------------------------------------------------------------- */
/* ARemSP scan (Algorithm 6) over rows [r0, r1): two rows and one column    */
/* per step with the mask of Fig. 1b: a b c / d e / f g, where e=(r,c),     */
/* g=(r+1,c), f=(r+1,c-1).  Rows outside [r0, r1) are treated as           */
/* background, which is what a chunk of Algorithm 7 sees.  Labels are      */
/* handed out from *count upward.                                           */
/* ---------------------------------------------------------------------- */
static void new_label(int32_t *lx, int32_t *p, int32_t *count)
{
    *lx = *count;
    p[*count] = *count;
    (*count)++;
}

static void scan_aremsp_rows(const image_t *im, int conn, int64_t r0, int64_t r1,
                             int32_t *label, int32_t *p, int32_t *count)
{
    for (int64_t r = r0; r < r1; r++)
        for (int64_t c = 0; c < im->W; c++)
            label[r * im->W + c] = 0;
    for (int64_t r = r0; r < r1; r += 2) {
        int has_g_row = (r + 1 < r1);
        for (int64_t c = 0; c < im->W; c++) {
            int in_up = (r - 1 >= r0);
            int e = image_at(im, r, c);
            int g = has_g_row ? image_at(im, r + 1, c) : 0;
            int a = in_up ? image_at(im, r - 1, c - 1) : 0;
            int b = in_up ? image_at(im, r - 1, c) : 0;
            int cc = in_up ? image_at(im, r - 1, c + 1) : 0;
            int d = image_at(im, r, c - 1);
            int f = has_g_row ? image_at(im, r + 1, c - 1) : 0;
            int32_t *le = &label[r * im->W + c];
            int32_t *lg = has_g_row ? &label[(r + 1) * im->W + c] : NULL;
            int32_t la = a ? label[(r - 1) * im->W + c - 1] : 0;
            int32_t lb = b ? label[(r - 1) * im->W + c] : 0;
            int32_t lc = cc ? label[(r - 1) * im->W + c + 1] : 0;
            int32_t ld = d ? label[r * im->W + c - 1] : 0;
            int32_t lf = f ? label[(r + 1) * im->W + c - 1] : 0;
            if (conn == 8) {
                if (e) {
                    if (!d) {
                        if (b) {
                            *le = lb;
                            if (f)
                                merge(p, *le, lf);
                        } else if (f) {
                            *le = lf;
                            if (a)
                                merge(p, *le, la);
                            if (cc)
                                merge(p, *le, lc);
                        } else if (a) {
                            *le = la;
                            if (cc)
                                merge(p, *le, lc);
                        } else if (cc) {
                            *le = lc;
                        } else {
                            new_label(le, p, count);
                        }
                    } else {
                        *le = ld;
                        if (!b && cc)
                            merge(p, *le, lc);
                    }
                    if (g)
                        *lg = *le;
                } else if (g) {
                    if (d)
                        *lg = ld;
                    else if (f)
                        *lg = lf;
                    else
                        new_label(lg, p, count);
                }
            } else {
                /* 4-connectivity: e sees b and d; g sees e and f. */
                if (e) {
                    if (b && d) {
                        *le = lb;
                        merge(p, *le, ld);
                    } else if (b) {
                        *le = lb;
                    } else if (d) {
                        *le = ld;
                    } else {
                        new_label(le, p, count);
                    }
                    if (g) {
                        *lg = *le;
                        if (f)
                            merge(p, *lg, lf);
                    }
                } else if (g) {
                    if (f)
                        *lg = lf;
                    else
                        new_label(lg, p, count);
                }
            }
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Canonical numbering: the k-th distinct nonzero label met in raster      */
/* order becomes k.  This is the numbering the GPU library promises:        */
/* components ranked by their smallest raster index.                        */
/* ---------------------------------------------------------------------- */
static int64_t canonical_numbering(int32_t *label, int64_t H, int64_t W, int32_t maxlabel)
{
    int32_t *map = (int32_t *)calloc((size_t)maxlabel + 1, sizeof(int32_t));
    if (!map)
        return -1;
    int32_t next = 1;
    for (int64_t i = 0; i < H * W; i++) {
        int32_t l = label[i];
        if (l == 0)
            continue;
        if (map[l] == 0)
            map[l] = next++;
        label[i] = map[l];
    }
    free(map);
    return next - 1;
}

/* ---------------------------------------------------------------------- */
/* Gray-level scan.  The already-scanned neighbours of e (a, b, c, d of     */
/* Fig. 1a under 8-connectivity, b and d under 4) whose byte equals e's     */
/* byte are merged with Algorithm 2; e takes a member of their united set,  */
/* or a new label when none has e's value.  Labels are handed out in raster */
/* order and every set's root is its smallest label, so the flatten         */
/* numbering is canonical.  Returns the largest label handed out.           */
/* ---------------------------------------------------------------------- */
static int32_t scan_gray(const image_t *im, int conn, int32_t *label, int32_t *p)
{
    static const int nb8[4][2] = {{-1, -1}, {-1, 0}, {-1, 1}, {0, -1}};
    static const int nb4[2][2] = {{-1, 0}, {0, -1}};
    const int (*nb)[2] = conn == 8 ? nb8 : nb4;
    const int nn = conn == 8 ? 4 : 2;
    int32_t count = 1;
    p[0] = 0;
    for (int64_t r = 0; r < im->H; r++) {
        for (int64_t c = 0; c < im->W; c++) {
            int32_t *e = &label[r * im->W + c];
            const uint8_t v = im->img[r * im->stride + c];
            *e = 0;
            if (v == 0)
                continue;
            int32_t l = 0;
            for (int k = 0; k < nn; k++) {
                const int64_t rr = r + nb[k][0], cc = c + nb[k][1];
                if (rr < 0 || cc < 0 || cc >= im->W || im->img[rr * im->stride + cc] != v)
                    continue;
                const int32_t ln = label[rr * im->W + cc];
                l = l ? merge(p, l, ln) : p[ln];
            }
            if (!l) {
                l = count;
                p[count] = count;
                count++;
            }
            *e = l;
        }
    }
    return count - 1;
}

/* ====================================================================== */
/* Exported entry points.  All return the number of components K >= 0, or  */
/* -1 on an argument or allocation error.  labels is a dense H x W int32    */
/* array (row pitch W); img has row pitch stride bytes.                    */
/* ====================================================================== */

static int bad_args(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int conn,
                    const int32_t *labels)
{
    return !img || !labels || H <= 0 || W <= 0 || stride < W || (conn != 4 && conn != 8) ||
           H * W >= INT32_MAX;
}

/* CCLRemSP (Algorithm 1): scan, flatten, labeling.  The scan hands out     */
/* labels in raster order and the set root is the smallest label, so the   */
/* flatten numbering is already canonical.                                  */
int64_t oracle_cclremsp(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int conn,
                        int32_t *labels)
{
    if (bad_args(img, H, W, stride, conn, labels))
        return -1;
    image_t im = {img, H, W, stride};
    int32_t *p = (int32_t *)malloc((size_t)max_labels(H, W) * sizeof(int32_t));
    if (!p)
        return -1;
    int32_t count = scan_cclremsp(&im, conn, labels, p);
    int32_t k = flatten(p, count);
    labeling_phase(labels, &im, p);
    free(p);
    return k;
}

/* Gray-level labeling: scan_gray, flatten, labeling.  Any two 4-adjacent  */
/* pixels may hold different values, so up to H*W labels are handed out.   */
int64_t oracle_gray(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int conn, int32_t *labels)
{
    if (bad_args(img, H, W, stride, conn, labels))
        return -1;
    image_t im = {img, H, W, stride};
    int32_t *p = (int32_t *)malloc((size_t)(H * W + 2) * sizeof(int32_t));
    if (!p)
        return -1;
    int32_t count = scan_gray(&im, conn, labels, p);
    int32_t k = flatten(p, count);
    labeling_phase(labels, &im, p);
    free(p);
    return k;
}

/* ARemSP (Algorithm 5) followed by the canonical numbering.  If raw is     */
/* nonzero the paper's own flatten numbering is kept instead.               */
int64_t oracle_aremsp(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int conn,
                      int32_t *labels, int raw)
{
    if (bad_args(img, H, W, stride, conn, labels))
        return -1;
    image_t im = {img, H, W, stride};
    int32_t *p = (int32_t *)malloc((size_t)max_labels(H, W) * sizeof(int32_t));
    if (!p)
        return -1;
    int32_t count = 1;
    p[0] = 0;
    scan_aremsp_rows(&im, conn, 0, H, labels, p, &count);
    int32_t k = flatten(p, count - 1);
    labeling_phase(labels, &im, p);
    free(p);
    if (!raw)
        return canonical_numbering(labels, H, W, k);
    return k;
}

/* PARemSP (Algorithm 7) with nchunks row chunks, followed by the canonical */
/* numbering.  Chunk k covers rows [start_k, start_{k+1}) where start_k =   */
/* 2*k*floor(ceil(H/2)/nchunks) and the last chunk takes the remainder.      */
int64_t oracle_paremsp(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int conn,
                       int32_t *labels, int nchunks)
{
    if (bad_args(img, H, W, stride, conn, labels) || nchunks <= 0)
        return -1;
    image_t im = {img, H, W, stride};
    int64_t numiter = (H + 1) / 2;
    if (nchunks > numiter)
        nchunks = (int)numiter;
    int64_t chunk = numiter / nchunks;
    int64_t size = 2 * chunk;
    /* Labels of chunk k live in [start*W + 1, start*W + rows*W], disjoint. */
    int64_t nlab = H * W + 2;
    int32_t *p = (int32_t *)malloc((size_t)nlab * sizeof(int32_t));
    if (!p)
        return -1;
    /* Labels never handed out map to background in flatten (p[i] = 0 < i). */
    for (int64_t i = 0; i < nlab; i++)
        p[i] = 0;
    int32_t maxlabel = 0;
    for (int k = 0; k < nchunks; k++) {
        int64_t start = (int64_t)k * size;
        int64_t end = (k == nchunks - 1) ? H : start + size;
        int32_t count = (int32_t)(start * W + 1);
        scan_aremsp_rows(&im, conn, start, end, labels, p, &count);
        if (count - 1 > maxlabel)
            maxlabel = count - 1;
    }
    /* Boundary merge: each chunk's first row against the previous chunk's  */
    /* last row, using label(x) != 0 as the foreground test.                */
    for (int64_t i = size; i < H && i <= (int64_t)(nchunks - 1) * size; i += size) {
        for (int64_t c = 0; c < W; c++) {
            int32_t le = labels[i * W + c];
            if (le == 0)
                continue;
            int32_t lb = label_at(labels, &im, i - 1, c);
            if (lb != 0) {
                merger(p, le, lb);
            } else if (conn == 8) {
                int32_t la = label_at(labels, &im, i - 1, c - 1);
                int32_t lc = label_at(labels, &im, i - 1, c + 1);
                if (la != 0)
                    merger(p, le, la);
                if (lc != 0)
                    merger(p, le, lc);
            }
        }
    }
    int32_t k = flatten(p, maxlabel);
    labeling_phase(labels, &im, p);
    free(p);
    return canonical_numbering(labels, H, W, k);
}

/* Canonical renumbering of an arbitrary labeling (0 = background).         */
/*
 * Provisional order: the numbering of the flatten (Algorithm 3) when the
 * provisional labels come from a tiled scan -- tiles of th x tw pixels in
 * raster order, each handing out its labels after those of the tiles before
 * it (Algorithm 7's per-partition label ranges, with tiles for row chunks),
 * and inside a tile one label per tile-local component, given in the order of
 * the component's first node, the nodes being runs of `block` rows ordered
 * by (block row, first column).  The smallest provisional label of a set is
 * then the minimum over its pixels of (tile index, block row inside the
 * tile, column inside the tile); the flatten numbers the sets 1..K in the
 * order of those minima.  `labels` holds any labeling 1..K of the partition
 * (0 = background); it is renumbered in place.  Returns K, or -1.
 */
static const int64_t *g_first; /* qsort context: smallest key of each set */
static int by_first(const void *a, const void *b)
{
    const int64_t x = g_first[*(const int32_t *)a], y = g_first[*(const int32_t *)b];
    return (x > y) - (x < y);
}

int64_t oracle_provisional(int32_t *labels, int64_t H, int64_t W, int64_t K, int th, int tw, int block)
{
    if (!labels || H <= 0 || W <= 0 || K < 0 || th <= 0 || tw <= 0 || block <= 0 || th % block)
        return -1;
    int64_t *first = malloc(sizeof(int64_t) * (size_t)(K + 1));
    int32_t *order = malloc(sizeof(int32_t) * (size_t)(K + 1));
    int32_t *rank = malloc(sizeof(int32_t) * (size_t)(K + 1));
    if (!first || !order || !rank) {
        free(first);
        free(order);
        free(rank);
        return -1;
    }
    const int64_t ntx = (W + tw - 1) / tw;
    for (int64_t k = 0; k <= K; k++)
        first[k] = INT64_MAX;
    for (int64_t r = 0; r < H; r++)
        for (int64_t c = 0; c < W; c++) {
            const int32_t g = labels[r * W + c];
            if (g <= 0)
                continue;
            const int64_t tile = (r / th) * ntx + c / tw;
            const int64_t key = tile * (int64_t)th * tw + ((r % th) / block) * tw + c % tw;
            if (key < first[g])
                first[g] = key;
        }
    for (int64_t k = 0; k < K; k++)
        order[k] = (int32_t)(k + 1);
    g_first = first;
    qsort(order, (size_t)K, sizeof(int32_t), by_first);
    for (int64_t k = 0; k < K; k++)
        rank[order[k]] = (int32_t)(k + 1);
    for (int64_t i = 0; i < H * W; i++)
        if (labels[i] > 0)
            labels[i] = rank[labels[i]];
    free(first);
    free(order);
    free(rank);
    return K;
}

int64_t oracle_canonical(int32_t *labels, int64_t H, int64_t W)
{
    int32_t maxlabel = 0;
    for (int64_t i = 0; i < H * W; i++)
        if (labels[i] > maxlabel)
            maxlabel = labels[i];
    return canonical_numbering(labels, H, W, maxlabel);
}

/* Expose Algorithm 2 and Algorithm 3 on a caller-owned parent array so the */
/* tests can check their invariants directly.  pairs holds m (x, y) pairs. */
void oracle_merge_pairs(int32_t *p, const int32_t *pairs, int64_t m)
{
    for (int64_t i = 0; i < m; i++)
        merge(p, pairs[2 * i], pairs[2 * i + 1]);
}

void oracle_merger_pairs(int32_t *p, const int32_t *pairs, int64_t m)
{
    for (int64_t i = 0; i < m; i++)
        merger(p, pairs[2 * i], pairs[2 * i + 1]);
}

int32_t oracle_flatten(int32_t *p, int32_t count)
{
    return flatten(p, count);
}
