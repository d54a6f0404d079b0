"""Comparison helpers shared by the tests (no method arithmetic)."""
import numpy as np


def fro_of_product(A, B):
    """||A B^T||_F from thin QR factors, without forming A B^T."""
    if A.shape[1] == 0:
        return 0.0
    Ra = np.linalg.qr(A, mode="r")
    Rb = np.linalg.qr(B, mode="r")
    return float(np.linalg.norm(Ra @ Rb.T))


def rel_diff_factored(Ua, Va, Ub, Vb):
    """||Ua Va^T - Ub Vb^T||_F / ||Ub Vb^T||_F (no cancellation of squares)."""
    num = fro_of_product(np.hstack([Ua, -Ub]), np.hstack([Va, Vb]))
    den = fro_of_product(Ub, Vb)
    return num / den if den > 0 else num


def gpu_case(name):
    """Print (and flush) which GPU case runs next, so a crash names it."""
    print(f"[gpu case] {name}", flush=True)
