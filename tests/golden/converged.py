"""Reader for the stored FP64 oracle mass flows of converged channel solves
(sweep_d2v37_converged.txt, serve_sample_converged.txt; written by
make_converged_golden.py, which calls only the oracle)."""
from pathlib import Path

HERE = Path(__file__).resolve().parent
SWEEP = HERE / "sweep_d2v37_converged.txt"
SERVE = HERE / "serve_sample_converged.txt"


def load_converged(path):
    """{key: dict(dvm, ny, kn, stop, mdot={step: value})} in file order."""
    out = {}
    cur = None
    for line in Path(path).read_text().splitlines():
        if not line or line.startswith("#"):
            continue
        t = line.split()
        if t[0] == "solve":
            cur = dict(dvm=t[2], ny=int(t[3]), kn=float(t[4]),
                       stop=None if t[5] == "None" else int(t[5]), mdot={})
            out[int(t[1])] = cur
        else:
            cur["mdot"][int(t[1])] = float(t[2])
    return out


def rel_err_at(entry, steps, mdot):
    """Relative error of a mass flow taken after `steps` steps against the
    oracle's value at the same step (None if the step is outside the stored
    window)."""
    want = entry["mdot"].get(int(steps))
    return None if want is None else abs(mdot - want) / abs(want)
