"""Reader for the DVM tables transcribed from the paper's appendices."""
from pathlib import Path

HERE = Path(__file__).resolve().parent


def load_dvm_tables(path=HERE / "dvm_tables.txt"):
    models = []
    cur = None
    for line in path.read_text().splitlines():
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        tok = line.split()
        if tok[0] == "model":
            cur = dict(label=tok[1], D=int(tok[2]), V=int(tok[3]), Q=int(tok[4]),
                       E=int(tok[5]), c=float(tok[6]), c_text=tok[6], table=tok[7],
                       kind=tok[8], gens=[], sizes=[], weights=[])
            models.append(cur)
        else:
            d = cur["D"]
            cur["gens"].append(tuple(int(t) for t in tok[:d]))
            cur["sizes"].append(int(tok[d]))
            cur["weights"].append(float(tok[d + 1]))
    return models
