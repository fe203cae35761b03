"""Step-level parity of a GPU step whose dipolar field is summed in reduced precision.

The check splits the step in two. The field: the Eq. 1 part of the GPU's total field
against the oracle's exact sum, as a relative Frobenius error. The rest of the step
(working plane, extrema, fall, Eq. 5, draw, new moment), which runs in FP64 on both
sides: the oracle's step fed the GPU's own total field must reproduce the GPU's
switching probabilities and moments to rounding. A jump decision may then differ from
the exact-field oracle's only where the draw u lies between the probability of the
exact field and that of the GPU's field."""
import numpy as np

from oracle import kmc


def check_reduced_step(pos, axes, m_in, k, p, seed, stream, diag_r, m_gpu, field_tol):
    """diag_r: the GPU's n x 8 diagnostics of the step (total field, P, jump flag);
    m_gpu: its new moments. Returns (field error, decisions that differ)."""
    m_new, info = kmc.step(pos, axes, m_in, k, p, seed, stream)
    Bg = diag_r[:, :3]
    eh = kmc.field_unit(p)
    dip_gpu = Bg - kmc.applied_field(k, p) * eh[None, :]
    err = np.linalg.norm(dip_gpu - info.Bdip) / np.linalg.norm(info.Bdip)
    assert err < field_tol, err
    m_own, own = kmc.step(pos, axes, m_in, k, p, seed, stream, B_override=Bg)
    assert np.abs(diag_r[:, 3] - own.P).max() < 1e-12
    jump_gpu = diag_r[:, 4] == 1.0
    same_own = jump_gpu == own.jump
    assert np.all((np.abs(own.u - own.P) < 1e-12)[~same_own])
    assert np.abs(m_gpu[same_own] - m_own[same_own]).max() < 1e-10
    dif = jump_gpu != info.jump
    band = np.abs(own.P - info.P) + 1e-12
    assert np.all((np.abs(info.u - info.P) <= band)[dif]), np.count_nonzero(dif)
    return err, int(np.count_nonzero(dif))
