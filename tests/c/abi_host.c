/* A plain C99 caller of libpbng's host-only entry points (no GPU needed):
 * the version, the Lame conversion of Eq. (lame), and the node colouring
 * of a single tetrahedron and of a two-triangle square.  Prints one line
 * per check and returns non-zero on the first failure. */
#include <math.h>
#include <stdio.h>

#include "pbng.h"
#include "pbng2d.h"

#define CHECK(c, msg)                                  \
    do {                                               \
        if (!(c)) {                                    \
            printf("FAIL %s: %s\n", msg, pbng_last_error()); \
            return 1;                                  \
        }                                              \
        printf("ok %s\n", msg);                        \
    } while (0)

int main(void)
{
    CHECK(pbng_version() == PBNG_ABI_VERSION, "version");

    double E = 1.0e4, nu = 0.25, mu = 0.0, lam = 0.0;
    CHECK(pbng_lame(1, &E, &nu, &mu, &lam) == PBNG_OK, "lame status");
    CHECK(fabs(mu - 4000.0) < 1e-9 && fabs(lam - 4000.0) < 1e-9, "lame values");
    nu = 0.5;
    CHECK(pbng_lame(1, &E, &nu, &mu, &lam) == PBNG_EINVAL, "lame rejects nu = 0.5");

    /* one tet, vertex 0 prescribed: the three free vertices take colours 0, 1, 2 */
    const double X[12] = {0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 1};
    const int32_t tet[4] = {0, 1, 2, 3};
    const int32_t didx[1] = {0};
    const double dx[3] = {0, 0, 0};
    pbng_problem p = {0};
    p.n_verts = 4;
    p.n_tets = 1;
    p.rest_pos = X;
    p.tets = tet;
    p.model = PBNG_NEOHOOKEAN;
    p.mu = 1.0;
    p.lambda = 1.0;
    p.n_dirichlet = 1;
    p.dirichlet_idx = didx;
    p.dirichlet_x = dx;
    int32_t col[4], nc = 0;
    CHECK(pbng_color(&p, col, &nc) == PBNG_OK, "tet colour status");
    CHECK(nc == 3 && col[0] == -1 && col[1] == 0 && col[2] == 1 && col[3] == 2, "tet colours");
    const int32_t bad[4] = {0, 1, 2, 7};
    p.tets = bad;
    CHECK(pbng_color(&p, col, &nc) == PBNG_EMESH, "tet index out of range");

    /* unit square, two counter-clockwise triangles, nothing prescribed */
    const double Y[8] = {0, 0, 1, 0, 0, 1, 1, 1};
    const int32_t tri[6] = {0, 1, 3, 0, 3, 2};
    pbng2d_problem q = {0};
    q.n_verts = 4;
    q.n_tris = 2;
    q.rest_pos = Y;
    q.tris = tri;
    q.model = PBNG_COROTATED;
    q.mu = 1.0;
    q.lambda = 1.0;
    CHECK(pbng2d_color(&q, col, &nc) == PBNG_OK, "square colour status");
    CHECK(nc == 3 && col[0] == 0 && col[1] == 1 && col[2] == 1 && col[3] == 2, "square colours");
    q.model = PBNG_STABLE_NEOHOOKEAN;
    CHECK(pbng2d_color(&q, col, &nc) == PBNG_EUNSUPPORTED, "planar stable Neo-Hookean rejected");
    return 0;
}
