/*
 * Runs the oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (built by tests/test_oracle_sanitize.py with gcc; host code only).
 *
 * Every labeling the oracle exports is compared with a textbook breadth-first
 * flood fill started at each unvisited object pixel in raster order, which
 * numbers components by their smallest raster index by construction:
 *   - every binary image with H*W <= 16 (all shapes), 4- and 8-connectivity,
 *     through CCLRemSP, ARemSP (canonical and raw) and PARemSP on 1..4 chunks;
 *   - random binary images of ragged shapes and densities;
 *   - random few-valued images through the gray-level labeling;
 *   - Algorithm 2 merges and Algorithm 3 flatten on random pair lists
 *     (p[i] <= i, roots are set minima, consecutive numbering).
 * Any mismatch prints the case and exits with status 1; a memory or
 * undefined-behaviour error aborts through the sanitizers.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t oracle_cclremsp(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int conn, int32_t *labels);
int64_t oracle_aremsp(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int conn, int32_t *labels,
                      int raw);
int64_t oracle_paremsp(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int conn, int32_t *labels,
                       int nchunks);
int64_t oracle_gray(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int conn, int32_t *labels);
int64_t oracle_canonical(int32_t *labels, int64_t H, int64_t W);
void oracle_merge_pairs(int32_t *p, const int32_t *pairs, int64_t m);
int64_t oracle_provisional(int32_t *labels, int64_t H, int64_t W, int64_t K, int th, int tw, int block);
int32_t oracle_flatten(int32_t *p, int32_t count);

static uint64_t rng_state = 0x1234567887654321ull;
static uint32_t rnd(void)
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (uint32_t)(rng_state >> 16);
}

/* Flood fill: pixels connect when both are nonzero and (gray) equal. */
static int64_t flood(const uint8_t *img, int H, int W, int conn, int gray, int32_t *lab, int32_t *queue)
{
    int64_t k = 0;
    memset(lab, 0, sizeof(int32_t) * (size_t)H * (size_t)W);
    for (int r = 0; r < H; r++)
        for (int c = 0; c < W; c++) {
            if (!img[r * W + c] || lab[r * W + c])
                continue;
            k++;
            int head = 0, tail = 0;
            queue[tail++] = r * W + c;
            lab[r * W + c] = (int32_t)k;
            while (head < tail) {
                const int v = queue[head++], vr = v / W, vc = v % W;
                for (int dr = -1; dr <= 1; dr++)
                    for (int dc = -1; dc <= 1; dc++) {
                        if ((dr == 0 && dc == 0) || (conn == 4 && dr != 0 && dc != 0))
                            continue;
                        const int nr = vr + dr, nc = vc + dc;
                        if (nr < 0 || nr >= H || nc < 0 || nc >= W)
                            continue;
                        const int u = nr * W + nc;
                        if (!img[u] || lab[u])
                            continue;
                        if (gray && img[u] != img[v])
                            continue;
                        lab[u] = (int32_t)k;
                        queue[tail++] = u;
                    }
            }
        }
    return k;
}

static int fails = 0;

static void expect_same(const char *what, const int32_t *got, int64_t kgot, const int32_t *ref, int64_t kref,
                        int H, int W, int conn)
{
    if (kgot != kref || memcmp(got, ref, sizeof(int32_t) * (size_t)H * (size_t)W) != 0) {
        if (fails < 10)
            fprintf(stderr, "%s differs from flood fill: H=%d W=%d conn=%d K=%lld vs %lld\n", what, H, W, conn,
                    (long long)kgot, (long long)kref);
        fails++;
    }
}

static void check_binary(const uint8_t *img, int H, int W, int32_t *ref, int32_t *got, int32_t *queue)
{
    for (int conn = 4; conn <= 8; conn += 4) {
        const int64_t kref = flood(img, H, W, conn, 0, ref, queue);
        int64_t k = oracle_cclremsp(img, H, W, W, conn, got);
        expect_same("cclremsp", got, k, ref, kref, H, W, conn);
        k = oracle_aremsp(img, H, W, W, conn, got, 0);
        expect_same("aremsp", got, k, ref, kref, H, W, conn);
        k = oracle_aremsp(img, H, W, W, conn, got, 1);
        if (k != kref)
            expect_same("aremsp raw count", got, k, ref, kref, H, W, conn);
        k = oracle_canonical(got, H, W);
        expect_same("aremsp raw renumbered", got, k, ref, kref, H, W, conn);
        for (int t = 1; t <= 4; t++) {
            k = oracle_paremsp(img, H, W, W, conn, got, t);
            expect_same("paremsp", got, k, ref, kref, H, W, conn);
        }
        /* provisional renumbering: a permutation of 1..K that renumbers back */
        memcpy(got, ref, sizeof(int32_t) * (size_t)H * (size_t)W);
        k = oracle_provisional(got, H, W, kref, 2, 3, conn == 8 ? 2 : 1);
        if (k == kref) {
            k = oracle_canonical(got, H, W);
            expect_same("provisional renumbered", got, k, ref, kref, H, W, conn);
        } else {
            expect_same("provisional count", got, k, ref, kref, H, W, conn);
        }
    }
}

int main(void)
{
    const int MAXPX = 1 << 20;
    uint8_t *img = malloc(MAXPX);
    int32_t *ref = malloc(sizeof(int32_t) * MAXPX), *got = malloc(sizeof(int32_t) * MAXPX);
    int32_t *queue = malloc(sizeof(int32_t) * MAXPX);
    if (!img || !ref || !got || !queue)
        return 2;
    long long cases = 0;
    /* every binary image of every shape with at most 16 pixels */
    for (int H = 1; H <= 16; H++)
        for (int W = 1; H * W <= 16; W++) {
            const int n = H * W;
            for (uint32_t bits = 0; bits < (1u << n); bits++) {
                for (int i = 0; i < n; i++)
                    img[i] = (uint8_t)((bits >> i) & 1u);
                check_binary(img, H, W, ref, got, queue);
                cases++;
            }
        }
    /* random images of ragged shapes */
    static const int shapes[][2] = {{1, 777}, {777, 1}, {2, 513}, {63, 65}, {128, 129}, {300, 301}, {1000, 997}};
    for (size_t s = 0; s < sizeof(shapes) / sizeof(shapes[0]); s++)
        for (int q = 1; q <= 9; q += 2) {
            const int H = shapes[s][0], W = shapes[s][1];
            for (int i = 0; i < H * W; i++)
                img[i] = (uint8_t)((rnd() % 10) < (uint32_t)q ? 1 + rnd() % 255 : 0);
            check_binary(img, H, W, ref, got, queue);
            cases++;
        }
    /* gray levels: few values so that equal neighbours are common */
    for (int t = 0; t < 2000; t++) {
        const int H = 1 + (int)(rnd() % 40), W = 1 + (int)(rnd() % 40), v = 2 + (int)(rnd() % 3);
        for (int i = 0; i < H * W; i++)
            img[i] = (uint8_t)(rnd() % (uint32_t)v);
        for (int conn = 4; conn <= 8; conn += 4) {
            const int64_t kref = flood(img, H, W, conn, 1, ref, queue);
            const int64_t k = oracle_gray(img, H, W, W, conn, got);
            expect_same("gray", got, k, ref, kref, H, W, conn);
        }
        cases++;
    }
    /* Algorithm 2 and 3 on random pair lists */
    for (int t = 0; t < 2000; t++) {
        const int n = 2 + (int)(rnd() % 300), m = (int)(rnd() % 400);
        int32_t *p = malloc(sizeof(int32_t) * (size_t)n), *pr = malloc(sizeof(int32_t) * 2 * (size_t)(m + 1));
        for (int i = 0; i < n; i++)
            p[i] = i;
        for (int j = 0; j < 2 * m; j++)
            pr[j] = 1 + (int32_t)(rnd() % (uint32_t)(n - 1));
        oracle_merge_pairs(p, pr, m);
        for (int i = 0; i < n; i++)
            if (p[i] > i || p[i] < 0) {
                fprintf(stderr, "merge broke p[i] <= i\n");
                fails++;
                break;
            }
        const int32_t k = oracle_flatten(p, n - 1);
        int32_t seen = 0;
        for (int i = 1; i < n; i++) {
            if (p[i] < 1 || p[i] > seen + 1) {
                fprintf(stderr, "flatten numbering not consecutive\n");
                fails++;
                break;
            }
            if (p[i] == seen + 1)
                seen++;
        }
        if (seen != k) {
            fprintf(stderr, "flatten count %d vs %d\n", k, seen);
            fails++;
        }
        free(p);
        free(pr);
    }
    free(img);
    free(ref);
    free(got);
    free(queue);
    printf("%lld cases, %d failures\n", cases, fails);
    return fails ? 1 : 0;
}
