"""A reduced run of the synthetic accuracy study (the tester of Sect. 2 on stand-in inputs):
relerr (Eq. (relerr), multiples of eps) of the GPU path and of the oracle's recursive
algorithms A, H and Z against the exact norm, for U(0,1) and N(0,1) inputs of 2^22
elements in binary64 and binary32, three seeds each.  The paper observes errors below
3 eps for its recursive algorithms on such inputs (Sect. 2, Fig. 1); the single accumulator of
Theorem 1 is run beside them and reported, its error growing with n."""
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
vnp = pytest.importorskip("paper_2509_06220_amd")

import bench  # noqa: E402  (the study's input definitions)
import vnp_gen  # noqa: E402


@pytest.mark.parametrize("fmt", ["f64", "f32"])
@pytest.mark.parametrize("dist", ["U(0,1)", "N(0,1)"])
def test_recursive_algorithms_stay_below_3_eps(dist, fmt):
    n = 1 << 22
    worst = {}
    for seed in range(3):
        x = bench.study_input(vnp_gen, dist, fmt, seed, n)
        ex = oracle.exact_nrm2(x)
        vals = {"gpu": vnp.nrmf(torch.from_numpy(x).cuda()).item(), "A": oracle.nrmf(x, "A"),
                "H": oracle.nrmf(x, "H"), "Z": oracle.nrmf(x, "Z"), "acc": oracle.nrm_acc(x)}
        for k, v in vals.items():
            worst[k] = max(worst.get(k, 0.0), oracle.relerr(v, ex, fmt))
    print(f"{dist} {fmt} n=2^22, worst relerr over 3 seeds: " +
          ", ".join(f"{k} {v:.3f} eps" for k, v in worst.items()), flush=True)
    for k in ("gpu", "A", "H", "Z"):
        assert worst[k] < 3.0, (k, worst[k])
