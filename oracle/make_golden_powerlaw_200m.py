"""Writes tests/golden/powerlaw_200m_top100.npz: the oracle's top-100 singular values and left
vectors of the 200M-nonzero power-law matrix (4096 x 2^24, Zipf(1.2) rows, 256 column blocks,
1024 seeded rows emptied inside each of 128 seeded blocks; gen.powerlaw_200m()).

TEST INFRASTRUCTURE: calls only the oracle (the Gram route: FP64 sparse Gram of Eq. 2, cyclic
two-sided Jacobi, the rank-safe threshold with u_G = 2^-53, the sign rule) and the seeded
generator.  Nothing here touches the GPU library.  The file is keyed by the SHA-256 of the
generated colptr, rowidx and values bytes, so a test can tell whether its matrix is the one the
values belong to.  V is not stored (13 GB): a test forms the expected V columns from the stored
U and sigma by the back-projection identity V = A^T U Sigma^-1 on sampled columns.

Usage: python -m oracle.make_golden_powerlaw_200m [--out PATH]   (about 30 min on 8 cores)
"""
import argparse
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

K = 100


def csc_sha256(A) -> str:
    h = hashlib.sha256()
    for a in (A.colptr, A.rowidx, A.values):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def main():
    import oracle
    from paper_2009_09767_amd import gen

    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(ROOT, "tests", "golden", "powerlaw_200m_top100.npz"))
    args = ap.parse_args()
    t0 = time.time()
    A = gen.powerlaw_200m(progress=lambda m: print(m, flush=True))
    t_gen = time.time() - t0
    sha = csc_sha256(A)
    print(f"generated M={A.M} N={A.N} nnz={A.nnz} in {t_gen:.0f} s, sha256 {sha}", flush=True)
    t1 = time.time()
    ref = oracle.svd(A.M, A.N, A.colptr, A.rowidx, A.values, k=K, tol=0.0, method="gram",
                     u_gram=oracle.U_FP64, want_v=False, max_sweeps=60)
    t_svd = time.time() - t1
    print(f"oracle gram route: rank {ref.rank}, sweeps {ref.sweeps}, {t_svd:.0f} s", flush=True)
    rownnz = np.bincount(A.rowidx, minlength=A.M)
    np.savez(args.out, sigma=ref.sigma, U=ref.U, rank=np.int32(ref.rank), tau=np.float64(ref.tau),
             sweeps=np.int32(ref.sweeps), n_nonempty=np.int32(int(np.count_nonzero(rownnz))),
             M=np.int32(A.M), N=np.int64(A.N), nnz=np.int64(A.nnz), k=np.int32(K),
             csc_sha256=np.array(sha), seconds=np.float64(t_svd),
             method=np.array("oracle gram route (FP64 sparse Gram + cyclic Jacobi), u_G = 2^-53, tol = 0"))
    print(f"wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
