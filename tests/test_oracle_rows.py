"""The two row scalings of the linear-quadratic system (``inputs.make_problem``
rows="scaled" / "paper", eq. full_space_optimality_system and its symmetrized
form remarked at the end of Section 2): the collective smoother and the
multigrid hierarchy produce the same iterates in both, up to the adjoint's
weights (p~_j = zeta_j p_j), while the residual norms (and so the printed
stopping rule) differ."""
import numpy as np
import pytest

from paper_2302_13680_amd import inputs


def _pair(domain):
    kw = dict(M=3, sigma=0.7, decay=True, yd=inputs.paper_target(15), f=0.0, field="gaussian", corr_len2=0.5,
              domain=domain)
    ps = inputs.collocation_problem(15, 2, 1e-4, rows="scaled", **kw)
    pp = inputs.collocation_problem(15, 2, 1e-4, rows="paper", **kw)
    return ps, pp


@pytest.mark.parametrize("smoother,theta,domain", [("jacobi", 0.5, "lshape"), ("gs", 1.0, "square")])
def test_same_iterates_up_to_the_adjoint_weights(smoother, theta, domain):
    from oracle.oracle import Oracle
    ps, pp = _pair(domain)
    N, nn = ps.N, ps.n * ps.n
    zeta = np.asarray(ps.c) / np.asarray(pp.c)               # c_scaled = zeta_j h^2, c_paper = h^2
    assert np.allclose(zeta.sum(), 1.0)
    os_, op = Oracle(ps, theta=theta, smoother=smoother), Oracle(pp, theta=theta, smoother=smoother)
    xs = os_.vcycle(np.zeros(os_.vlen()), ps.rhs_paper(), 3)
    xp = op.vcycle(np.zeros(op.vlen()), pp.rhs_paper(), 3)
    ys, us, pts = xs[:N * nn], xs[N * nn:(N + 1) * nn], xs[(N + 1) * nn:].reshape(N, nn)
    yp, up, ptp = xp[:N * nn], xp[N * nn:(N + 1) * nn], xp[(N + 1) * nn:].reshape(N, nn)
    rel = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)
    assert rel(yp, ys) <= 1e-12 and rel(up, us) <= 1e-12
    assert rel(zeta[:, None] * ptp, pts) <= 1e-12           # p~_j = zeta_j p_j
    # the residual norms are weighted differently: the paper rows' Y residual is
    # 1/zeta_j times the scaled one
    rs, rp = os_.residual(xs, ps.rhs_paper()), op.residual(xp, pp.rhs_paper())
    ry_s, ry_p = rs[:N * nn].reshape(N, nn), rp[:N * nn].reshape(N, nn)
    assert rel(ry_p * zeta[:, None], ry_s) <= 1e-10
    assert not np.isclose(np.linalg.norm(rp) / np.linalg.norm(pp.rhs_paper()),
                          np.linalg.norm(rs) / np.linalg.norm(ps.rhs_paper()), rtol=1e-3)
