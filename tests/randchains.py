"""Random tiny loop chains for dependency and plan tests (neutral description:
plain dicts, converted to the oracle's or the library's types by the tests)."""
import random


def star_pts(ndim, r):
    pts = [tuple([0] * ndim)]
    for d in range(ndim):
        for s in range(-r, r + 1):
            if s:
                p = [0] * ndim
                p[d] = s
                pts.append(tuple(p))
    return pts


def random_chain(rng: random.Random, ndim: int, max_loops: int = 6):
    """Loops over random sub-ranges of a padded box, 1-3 datasets each,
    READ / WRITE / RW / INC access; write stencils are the centre only."""
    n = [rng.randint(4, 10) for _ in range(ndim)]
    ndat = rng.randint(2, 4)
    loops = []
    for _ in range(rng.randint(1, max_loops)):
        st = [rng.randint(-2, 2) for _ in range(ndim)]
        en = [max(n[d] + rng.randint(-2, 2), st[d]) for d in range(ndim)]
        dats = list(range(ndat))
        rng.shuffle(dats)
        args = []
        for a in dats[: rng.randint(1, min(3, ndat))]:
            acc = rng.choice(["R", "R", "W", "RW", "INC"])
            if acc == "R":
                sten = star_pts(ndim, rng.randint(0, 2))
                if rng.random() < 0.3:
                    sten = [tuple(rng.randint(-2, 2) for _ in range(ndim)) for _ in range(rng.randint(1, 3))]
            else:
                sten = [tuple([0] * ndim)]
            args.append({"dat": a, "stencil": sten, "access": acc})
        loops.append({"start": st, "end": en, "args": args})
    return {"ndim": ndim, "ndat": ndat, "n": n, "loops": loops}


def to_oracle(chain):
    from oracle.skewed import Arg, Loop
    return [Loop(list(l["start"]), list(l["end"]),
                 [Arg(a["dat"], [tuple(p) for p in a["stencil"]], a["access"]) for a in l["args"]])
            for l in chain["loops"]]
