"""Config 5 at full size (4096 x 2^24, ~200M nnz, 256 column blocks, mixed precision: FP32 Gram,
FP64 eigensolve and Rayleigh-Ritz, FP32 V, k = 100).  The oracle cannot finish this size, so the
checks are properties that hold at any size, against an FP64 product A^T U computed by torch's
own sparse matmul (independent of this library): sigma_i = ||A^T u_i||, V = A^T U Sigma^-1 with
unit columns, U^T U = I, the rank, and sigma sorted above tau."""
import numpy as np
import pytest

from paper_2009_09767_amd import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_09767_amd import ranky

    ranky.lib()
    return ranky


def test_powerlaw_200m_full_size_properties(R):
    import torch

    A = gen.powerlaw_200m(progress=lambda m: print(m, flush=True))
    print(f"powerlaw_200m: M={A.M} N={A.N} nnz={A.nnz}", flush=True)
    dA = R.to_device(A)
    k, D = A.meta["k"], A.meta["D"]
    out = R.svd(dA, k, 0.0, n_blocks=D, gram_prec="fp32", refine=1, v_dtype=torch.float32)
    info = out.info
    print("info", {n: info[n] for n in ("status", "rank", "sweeps", "tau", "sigma_max")}, flush=True)
    assert info["status"] == R.OK
    assert info["n_nonempty"] == A.M          # rows are emptied inside blocks only
    assert info["rank"] == k
    sig = out.sigma.cpu().numpy()
    assert np.all(np.diff(sig) <= 0) and sig[-1] > info["tau"]
    U = out.U
    orth = (U.T @ U - torch.eye(k, dtype=torch.float64, device=U.device)).abs().max().item()
    assert orth <= 1e-10, orth
    # Z = A^T U in FP64 by torch's sparse matmul (A^T as CSR = A's CSC arrays)
    At = torch.sparse_csr_tensor(dA.colptr.long(), dA.rowidx.long(), dA.values.double(), size=(A.N, A.M))
    Z = torch.sparse.mm(At, U)
    znorm = torch.linalg.vector_norm(Z, dim=0).cpu().numpy()
    rel = np.max(np.abs(znorm - sig) / sig)
    print(f"max |sigma - ||A^T u||| / sigma = {rel:.3e}", flush=True)
    assert rel <= 1e-6                        # the mixed-precision bar
    Vref = Z / out.sigma
    verr = ((out.V.double() - Vref).abs().max(dim=0).values / Vref.abs().max(dim=0).values).max().item()
    vn = torch.linalg.vector_norm(out.V.double(), dim=0).cpu().numpy()
    print(f"V vs A^T U / sigma: {verr:.3e}; column norms in [{vn.min():.7f}, {vn.max():.7f}]", flush=True)
    assert verr <= 1e-5                       # FP32 V
    assert np.all(np.abs(vn - 1.0) <= 1e-5)
