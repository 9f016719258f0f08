/* A plain C99 caller of libpbng on the GPU, with no other binding: reads
 * one tetrahedral problem from a raw file, solves it through the C ABI in
 * FP64 (pbng_workspace_create, pbng_solve, pbng_residual) with device
 * memory from the HIP runtime, and writes the result for the caller to
 * check.  Usage: abi_gpu IN OUT SWEEPS.
 *
 * IN holds, in order: int32 n_verts, n_tets, n_dirichlet, model; double mu,
 * lambda; double rest_pos[n_verts][3]; int32 tets[n_tets][4]; int32
 * dirichlet_idx[n_dirichlet]; double dirichlet_x[n_dirichlet][3]; double
 * x0[n_verts][3].  OUT receives double x[n_verts][3], the FP64 residual
 * norm and the number of colours. */
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "pbng.h"

static int rd(void* p, size_t size, size_t n, FILE* f) { return fread(p, size, n, f) == n ? 0 : 1; }

int main(int argc, char** argv)
{
    if (argc != 4) {
        fprintf(stderr, "usage: abi_gpu IN OUT SWEEPS\n");
        return 2;
    }
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t hdr[4];
    double lame[2];
    if (rd(hdr, sizeof(int32_t), 4, f) || rd(lame, sizeof(double), 2, f)) return 2;
    const int32_t nv = hdr[0], nt = hdr[1], nd = hdr[2];
    double* X = malloc(sizeof(double) * 3 * (size_t)nv);
    int32_t* T = malloc(sizeof(int32_t) * 4 * (size_t)nt);
    int32_t* D = malloc(sizeof(int32_t) * (size_t)(nd > 0 ? nd : 1));
    double* XD = malloc(sizeof(double) * 3 * (size_t)(nd > 0 ? nd : 1));
    double* x0 = malloc(sizeof(double) * 3 * (size_t)nv);
    if (!X || !T || !D || !XD || !x0) return 2;
    if (rd(X, sizeof(double), 3 * (size_t)nv, f) || rd(T, sizeof(int32_t), 4 * (size_t)nt, f) ||
        rd(D, sizeof(int32_t), (size_t)nd, f) || rd(XD, sizeof(double), 3 * (size_t)nd, f) ||
        rd(x0, sizeof(double), 3 * (size_t)nv, f))
        return 2;
    fclose(f);

    pbng_problem p = {0};
    p.n_verts = nv;
    p.n_tets = nt;
    p.rest_pos = X;
    p.tets = T;
    p.model = hdr[3];
    p.mu = lame[0];
    p.lambda = lame[1];
    p.n_dirichlet = nd;
    p.dirichlet_idx = D;
    p.dirichlet_x = XD;
    pbng_workspace* ws = NULL;
    if (pbng_workspace_create(&p, 1, NULL, PBNG_F64, &ws) != PBNG_OK) {
        fprintf(stderr, "create: %s\n", pbng_last_error());
        return 1;
    }
    double* xd = NULL;
    if (hipMalloc((void**)&xd, sizeof(double) * 3 * (size_t)nv) != hipSuccess) return 1;
    if (hipMemcpy(xd, x0, sizeof(double) * 3 * (size_t)nv, hipMemcpyHostToDevice) != hipSuccess) return 1;
    pbng_solve_opts o;
    pbng_default_solve_opts(&o);
    o.max_sweeps = atoi(argv[3]);
    o.rel_tol = 0.0;
    o.check_every = o.max_sweeps;
    o.accel = PBNG_ACCEL_NONE;
    o.safeguard = PBNG_SAFEGUARD_BACKTRACK;
    pbng_stats st;
    const int32_t rc = pbng_solve(ws, xd, &o, &st, NULL);
    if (rc != PBNG_OK && rc != PBNG_NOT_CONVERGED) {
        fprintf(stderr, "solve: %s\n", pbng_last_error());
        return 1;
    }
    double res = -1.0, energy = 0.0;
    if (pbng_residual(ws, xd, &res, &energy, NULL, NULL) != PBNG_OK) {
        fprintf(stderr, "residual: %s\n", pbng_last_error());
        return 1;
    }
    if (hipMemcpy(x0, xd, sizeof(double) * 3 * (size_t)nv, hipMemcpyDeviceToHost) != hipSuccess) return 1;
    FILE* g = fopen(argv[2], "wb");
    if (!g) return 2;
    const double ncol = st.n_colors;
    if (fwrite(x0, sizeof(double), 3 * (size_t)nv, g) != 3 * (size_t)nv || fwrite(&res, sizeof(double), 1, g) != 1 ||
        fwrite(&ncol, sizeof(double), 1, g) != 1)
        return 2;
    fclose(g);
    printf("sweeps %d colours %d residual %.6e\n", st.sweeps, st.n_colors, res);
    pbng_workspace_destroy(ws);
    (void)hipFree(xd);
    free(X);
    free(T);
    free(D);
    free(XD);
    free(x0);
    return 0;
}
