"""The seeded workload generators: determinism, ranges, boundary data."""
import hashlib

import numpy as np

import inputs


def _h(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_config0_deterministic_and_well_formed():
    a = inputs.config(0)
    b = inputs.config(0)
    assert _h(a.rho) == _h(b.rho) and _h(a.f) == _h(b.f)
    d = a.desc
    assert d["nel"] == (64, 32) and d["sub_nel"] == (16, 16) and d["overlap"] == 2
    assert inputs.n_dofs(d) == 4290
    assert a.rho.shape == (64 * 32,)
    assert set(np.unique(a.rho)) <= {0.0, 1.0}
    assert 0.3 < a.rho.mean() < 0.7
    assert a.fixed.sum() == 2 * 33          # left edge clamped
    assert np.all(a.f[a.fixed == 1] == 0)
    assert a.f.sum() == -1.0
    # load on solid material
    p = inputs.node_id(d, (64, 16))
    assert a.f[2 * p + 1] == -1.0
    assert a.rho[63 + 64 * 15] == 1.0 and a.rho[63 + 64 * 16] == 1.0


def test_config1_shapes():
    c = inputs.config(1)
    assert inputs.n_dofs(c.desc) == 263682
    assert c.fixed.sum() == 2 * 257
    assert c.desc["eig_kmax"] == inputs.KMAX_FRAGMENTED


def test_fill_hinges_leaves_no_diagonal_contacts_2d():
    rng = np.random.default_rng(0)
    rho = (rng.uniform(size=(40, 30)) < 0.3).astype(float)
    out = inputs.fill_hinges(rho) > 0.5
    a, b, c, d = out[:-1, :-1], out[1:, 1:], out[1:, :-1], out[:-1, 1:]
    assert not np.any(a & b & ~c & ~d)
    assert not np.any(c & d & ~a & ~b)
    assert np.all(out[rho > 0.5])


def test_fill_hinges_3d_face_connected_windows():
    rng = np.random.default_rng(1)
    rho = (rng.uniform(size=(10, 9, 8)) < 0.2).astype(float)
    s = inputs.fill_hinges(rho) > 0.5
    # in every 2x2x2 window the solid cells form one face-connected set
    for i in range(9):
        for j in range(8):
            for k in range(7):
                w = s[i:i + 2, j:j + 2, k:k + 2]
                cells = [tuple(c) for c in np.argwhere(w)]
                if len(cells) < 2:
                    continue
                seen = {cells[0]}
                stack = [cells[0]]
                while stack:
                    c = stack.pop()
                    for o in cells:
                        if o not in seen and sum(abs(x - y) for x, y in zip(c, o)) == 1:
                            seen.add(o)
                            stack.append(o)
                assert len(seen) == len(cells), (i, j, k)


def test_config_p_definition():
    p = inputs.config_p()
    assert p.desc["sub_mode"] == 1 and p.tol == 1e-6
    assert p.fixed.sum() == 2 * 400
    assert np.count_nonzero(p.f) == 2


def test_face_patch_load_total():
    desc = inputs.problem_desc(3, (8, 8, 8), sub_nel=4, overlap=1)
    f = inputs.face_patch_load(desc, 3, 6, 1, -1.0)
    assert abs(f.sum() + 1.0) < 1e-15
    assert np.count_nonzero(f) == 16
