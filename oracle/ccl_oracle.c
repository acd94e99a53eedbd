/*
 * CPU oracle for two-pass connected component labeling (Gupta, Palsetia,
 * Patwary, Agrawal, Choudhary, "A New Parallel Algorithm for Two-Pass
 * Connected Component Labeling", arXiv 1606.05973).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this file.  It shares no code with
 * the GPU library and must never be used as a fallback for it.
 *
 * Plain, slow C, single-threaded except for oracle_paremsp_threads.  Every
 * routine is written from the paper's description of the method, its steps
 * taken in the paper's order:
 *   merge        -- Rem's union with splicing (Section III, Algorithm 2)
 *   flatten      -- analysis phase (Section III, Algorithm 3)
 *   cclremsp     -- CCLRemSP: decision-tree scan (Fig. 2, Algorithm 4),
 *                   flatten, labeling phase (Algorithm 1)
 *   aremsp       -- ARemSP: two-row scan with the mask of Fig. 1b
 *                   (Algorithm 6), flatten, labeling (Algorithm 5)
 *   paremsp      -- PARemSP: chunked ARemSP scans with disjoint label
 *                   ranges, boundary-row merge with merger (Algorithms 7, 8),
 *                   flatten, labeling; the chunks either one after another
 *                   (oracle_paremsp) or one POSIX thread per chunk with the
 *                   boundary unions concurrent under Algorithm 8's locks
 *                   (oracle_paremsp_threads, the paper's parallel method as
 *                   a CPU baseline; checked under ThreadSanitizer)
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
#include <pthread.h>
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
/* Rem's union with splicing: the merge of Section III (Algorithm 2).       */
/* Parents only ever point to smaller labels (p[i] <= i), so the root of a  */
/* set is its smallest label.  The walk keeps one node on each side; at     */
/* every step the node whose parent is the larger one moves: if it is a     */
/* root it is hung below the other node's parent and the two sets are one;  */
/* otherwise it is spliced onto the other node's parent (a smaller label of */
/* the set being united) and the walk continues from its old parent.  The   */
/* walk ends when both nodes have the same parent.  The value returned is a */
/* member of the united set (a parent value, as in the paper), which is all */
/* the scan needs for the label of the current pixel.                       */
/* ---------------------------------------------------------------------- */
static int32_t merge(int32_t *p, int32_t x, int32_t y)
{
    for (;;) {
        int32_t px = p[x], py = p[y];
        if (px == py)
            return px;
        if (px < py) {
            /* the side that moves is called x */
            int32_t t = x;
            x = y;
            y = t;
            t = px;
            px = py;
            py = t;
        }
        p[x] = py; /* a root is linked, an inner node spliced */
        if (px == x)
            return py;
        x = px;
    }
}

/* ---------------------------------------------------------------------- */
/* The concurrent union of PARemSP's boundary phase (Section IV, the merger */
/* of Algorithm 8): Rem's union run by several threads on one parent array. */
/* Splices need no lock (the paper's memory model: each parent entry is     */
/* read and written whole, here as relaxed C11 atomics).  Hanging a root    */
/* below another set is done under the root's lock, after checking again,   */
/* under the lock, that the node is still a root; if another thread hung it */
/* meanwhile, the walk carries on from where it is.  Every store keeps      */
/* p[i] < i for an inner node, so the forest stays acyclic.  Locks are      */
/* striped: root x uses lk[x % nlk].  With lk == NULL (one thread) this is  */
/* the merge above step for step.                                           */
/* ---------------------------------------------------------------------- */
static int32_t ld(const int32_t *p, int32_t i)
{
    return __atomic_load_n(&p[i], __ATOMIC_RELAXED);
}

static void st(int32_t *p, int32_t i, int32_t v)
{
    __atomic_store_n(&p[i], v, __ATOMIC_RELAXED);
}

static void merger(int32_t *p, pthread_mutex_t *lk, int nlk, int32_t x, int32_t y)
{
    for (;;) {
        int32_t px = ld(p, x), py = ld(p, y);
        if (px == py)
            return;
        if (px < py) {
            int32_t t = x;
            x = y;
            y = t;
            t = px;
            px = py;
            py = t;
        }
        if (px == x) {
            int linked = 0;
            if (lk)
                pthread_mutex_lock(&lk[x % nlk]);
            if (ld(p, x) == x) {
                st(p, x, py);
                linked = 1;
            }
            if (lk)
                pthread_mutex_unlock(&lk[x % nlk]);
            if (linked)
                return;
            continue; /* no longer a root: look again from here */
        }
        st(p, x, py);
        x = px;
    }
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

/* Boundary step of PARemSP (Algorithm 7) for the chunk starting at row i:  */
/* every object pixel of row i (label(e) != 0 is the foreground test) is    */
/* united with its object neighbours in row i - 1, the last row of the      */
/* chunk above: b, else (8-connectivity) a and c.                           */
static void merge_boundary_row(const image_t *im, int conn, const int32_t *labels, int32_t *p,
                               pthread_mutex_t *lk, int nlk, int64_t i)
{
    const int64_t W = im->W;
    for (int64_t c = 0; c < W; c++) {
        int32_t le = labels[i * W + c];
        if (le == 0)
            continue;
        int32_t lb = label_at(labels, im, i - 1, c);
        if (lb != 0) {
            merger(p, lk, nlk, le, lb);
        } else if (conn == 8) {
            int32_t la = label_at(labels, im, i - 1, c - 1);
            int32_t lc = label_at(labels, im, i - 1, c + 1);
            if (la != 0)
                merger(p, lk, nlk, le, la);
            if (lc != 0)
                merger(p, lk, nlk, le, lc);
        }
    }
}

/* Chunking of Algorithm 7: H/2 row pairs dealt out in nchunks chunks of    */
/* size = 2 * floor(ceil(H/2) / nchunks) rows; the last chunk takes the     */
/* remainder; chunk k hands out labels from start*W + 1 (disjoint ranges,   */
/* none of them 0).                                                         */
typedef struct {
    const image_t *im;
    int conn;
    int32_t *labels, *p;
    int64_t start, end;   /* rows [start, end) */
    int32_t next_label;   /* in: first label of the chunk; out: one past its last */
    pthread_mutex_t *lk;
    int nlk;
} chunk_t;

static int plan_chunks(int64_t H, int nchunks, int64_t *size)
{
    int64_t numiter = (H + 1) / 2;
    if (nchunks > numiter)
        nchunks = (int)numiter;
    *size = 2 * (numiter / nchunks);
    return nchunks;
}

static void *chunk_scan(void *arg)
{
    chunk_t *ck = (chunk_t *)arg;
    scan_aremsp_rows(ck->im, ck->conn, ck->start, ck->end, ck->labels, ck->p, &ck->next_label);
    return NULL;
}

static void *chunk_boundary(void *arg)
{
    chunk_t *ck = (chunk_t *)arg;
    if (ck->start > 0)
        merge_boundary_row(ck->im, ck->conn, ck->labels, ck->p, ck->lk, ck->nlk, ck->start);
    return NULL;
}

static void *chunk_labeling(void *arg)
{
    chunk_t *ck = (chunk_t *)arg;
    const int64_t W = ck->im->W;
    for (int64_t i = ck->start * W; i < ck->end * W; i++)
        ck->labels[i] = ck->p[ck->labels[i]];
    return NULL;
}

/* Runs fn on every chunk: on its own thread each (threads = 1: one after   */
/* another on the caller's thread).  Returns -1 if a thread cannot start.   */
static int run_chunks(chunk_t *ck, int n, int threads, void *(*fn)(void *))
{
    if (!threads) {
        for (int k = 0; k < n; k++)
            fn(&ck[k]);
        return 0;
    }
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)n);
    if (!th)
        return -1;
    int started = 0, st = 0;
    for (; started < n; started++)
        if (pthread_create(&th[started], NULL, fn, &ck[started]) != 0) {
            st = -1;
            break;
        }
    for (int k = 0; k < started; k++)
        pthread_join(th[k], NULL);
    /* a chunk whose thread did not start is run here */
    for (int k = started; k < n; k++)
        fn(&ck[k]);
    free(th);
    return st;
}

/* PARemSP (Algorithm 7): scan the chunks (ARemSP, Algorithm 6), unite     */
/* across the chunk boundaries (merger, Algorithm 8), flatten (Algorithm 3) */
/* and the labeling phase, then the canonical numbering.  threads = 0: the  */
/* chunks one after another on the calling thread (one schedule the         */
/* concurrent algorithm admits); threads = 1: every phase's chunks on their */
/* own threads at once, the boundary unions concurrent under Algorithm 8's  */
/* locks.                                                                   */
static int64_t paremsp_run(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int conn, int32_t *labels,
                           int nchunks, int threads)
{
    if (bad_args(img, H, W, stride, conn, labels) || nchunks <= 0)
        return -1;
    image_t im = {img, H, W, stride};
    int64_t size;
    nchunks = plan_chunks(H, nchunks, &size);
    const int64_t nlab = H * W + 2;
    int32_t *p = (int32_t *)malloc((size_t)nlab * sizeof(int32_t));
    chunk_t *ck = (chunk_t *)calloc((size_t)nchunks, sizeof(chunk_t));
    const int nlk = 4096;
    pthread_mutex_t *lk = threads ? (pthread_mutex_t *)malloc(sizeof(pthread_mutex_t) * nlk) : NULL;
    if (!p || !ck || (threads && !lk)) {
        free(p);
        free(ck);
        free(lk);
        return -1;
    }
    for (int k = 0; k < (threads ? nlk : 0); k++)
        pthread_mutex_init(&lk[k], NULL);
    /* labels never handed out map to background in flatten (p[i] = 0 < i) */
    memset(p, 0, (size_t)nlab * sizeof(int32_t));
    for (int k = 0; k < nchunks; k++) {
        ck[k].im = &im;
        ck[k].conn = conn;
        ck[k].labels = labels;
        ck[k].p = p;
        ck[k].start = (int64_t)k * size;
        ck[k].end = (k == nchunks - 1) ? H : ck[k].start + size;
        ck[k].next_label = (int32_t)(ck[k].start * W + 1);
        ck[k].lk = lk;
        ck[k].nlk = nlk;
    }
    int st = run_chunks(ck, nchunks, threads, chunk_scan);
    if (st == 0)
        st = run_chunks(ck, nchunks, threads, chunk_boundary);
    int64_t k_out = -1;
    if (st == 0) {
        int32_t maxlabel = 0;
        for (int k = 0; k < nchunks; k++)
            if (ck[k].next_label - 1 > maxlabel)
                maxlabel = ck[k].next_label - 1;
        const int32_t k = flatten(p, maxlabel);
        st = run_chunks(ck, nchunks, threads, chunk_labeling);
        if (st == 0)
            k_out = canonical_numbering(labels, H, W, k);
    }
    for (int k = 0; k < (threads ? nlk : 0); k++)
        pthread_mutex_destroy(&lk[k]);
    free(lk);
    free(ck);
    free(p);
    return k_out;
}

/* PARemSP with nchunks row chunks run one after another; canonical         */
/* numbering.                                                               */
int64_t oracle_paremsp(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int conn, int32_t *labels,
                       int nchunks)
{
    return paremsp_run(img, H, W, stride, conn, labels, nchunks, 0);
}

/* PARemSP with one thread per chunk (POSIX threads; the CPU baseline of the */
/* paper's own parallel method); canonical numbering.                       */
int64_t oracle_paremsp_threads(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int conn,
                               int32_t *labels, int nthreads)
{
    return paremsp_run(img, H, W, stride, conn, labels, nthreads, 1);
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
        merger(p, NULL, 0, pairs[2 * i], pairs[2 * i + 1]);
}

int32_t oracle_flatten(int32_t *p, int32_t count)
{
    return flatten(p, count);
}
