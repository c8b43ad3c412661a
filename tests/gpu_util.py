"""Helpers shared by the GPU tests: device transfer and the parity rule."""

import numpy as np

import oracle

NCC_TOL = 1e-5  # absolute tolerance on NCC / confidence, and on the argmax gap


def to_dev(a: np.ndarray):
    import torch

    a = np.ascontiguousarray(a)
    if a.dtype == np.uint16:
        return torch.from_numpy(a.view(np.int16)).cuda().view(torch.uint16)
    return torch.from_numpy(a).cuda()


def to_host(t) -> np.ndarray:
    import torch

    if t.dtype == torch.uint16:
        return t.view(torch.int16).cpu().numpy().view(np.uint16)
    return t.cpu().numpy()


def check_match(ref, flt, centers, block, window, disp_g, ncc_g, conf_g, label=""):
    """The parity rule: a GPU displacement is accepted if it equals the
    oracle's, or if it is valid and its oracle NCC is within NCC_TOL of the
    oracle maximum; the reported NCC and confidence must match the oracle's
    NCC at the GPU displacement within NCC_TOL.  Returns (max argmax gap,
    max |ncc error|, number of non-identical displacements)."""
    srf = oracle.ncc_surface(ref, flt, centers, block, window)
    d_o, n_o, c_o = oracle.match(ref, flt, centers, block, window)
    gap_max = err_max = 0.0
    differ = 0
    for k in range(len(centers)):
        if np.isnan(n_o[k]):  # block not inside the volume
            assert np.isnan(ncc_g[k]) and conf_g[k] == 0 and np.all(disp_g[k] == 0), (label, k)
            continue
        dg = disp_g[k]
        assert np.all(np.abs(dg) <= window), (label, k, dg)
        v = srf[k, dg[2] + window, dg[1] + window, dg[0] + window]
        assert not np.isnan(v), ("GPU displacement invalid", label, k, dg)
        gap = n_o[k] - v
        assert gap < NCC_TOL, ("argmax gap", label, k, dg, d_o[k], gap)
        err = abs(float(ncc_g[k]) - v)
        assert err <= NCC_TOL, ("ncc", label, k, ncc_g[k], v)
        assert abs(float(conf_g[k]) - max(0.0, v)) <= NCC_TOL, ("conf", label, k)
        gap_max = max(gap_max, gap)
        err_max = max(err_max, err)
        differ += int(not np.array_equal(dg, d_o[k]))
    return gap_max, err_max, differ
