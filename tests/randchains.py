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


def random_op_chain(rng: random.Random, ndim: int, n=None, max_loops: int = 8, ndat: int = None, halo: int = 4):
    """Random chain of weighted-sum loops (one written dataset, 1-3 inputs
    read through random stencils) and axpby loops (one RW dataset, one read),
    over random sub-ranges of the padded box; representable both in the
    oracle and through the library's op vocabulary."""
    n = n or [rng.randint(5, 12) for _ in range(ndim)]
    ndat = ndat or rng.randint(3, 5)
    loops = []
    for _ in range(rng.randint(1, max_loops)):
        st = [rng.randint(-2, 1) for _ in range(ndim)]
        en = [max(n[d] + rng.randint(-1, 2), st[d]) for d in range(ndim)]
        dats = list(range(ndat))
        rng.shuffle(dats)
        if rng.random() < 0.75:
            k = rng.randint(1, min(3, ndat - 1))
            ins = []
            for a in dats[1:1 + k]:
                if rng.random() < 0.5:
                    sten = star_pts(ndim, rng.randint(0, 2))
                else:
                    sten = [tuple(rng.randint(-2, 2) for _ in range(ndim)) for _ in range(rng.randint(1, 4))]
                ins.append({"dat": a, "stencil": sten, "access": "R"})
            w = [rng.uniform(-0.5, 0.5) for a in ins for _ in a["stencil"]]
            loops.append({"op": "WSUM", "start": st, "end": en, "params": w,
                          "args": [{"dat": dats[0], "stencil": [tuple([0] * ndim)], "access": "W"}] + ins})
        else:
            loops.append({"op": "AXPBY", "start": st, "end": en,
                          "params": [rng.uniform(-1, 1), rng.uniform(-1, 1)],
                          "args": [{"dat": dats[0], "stencil": [tuple([0] * ndim)], "access": "RW"},
                                   {"dat": dats[1], "stencil": [tuple([0] * ndim)], "access": "R"}]})
    return {"ndim": ndim, "ndat": ndat, "n": n, "halo": halo, "loops": loops}


def op_chain_data(chain, seed: int):
    import numpy as np
    from synthgen import uniform_block
    shape = tuple(s + 2 * chain["halo"] for s in reversed(chain["n"]))
    size = int(np.prod(shape))
    return [uniform_block(seed, d * size, size, -1, 1).reshape(shape) for d in range(chain["ndat"])]


def run_op_chain_oracle(chain, data):
    """Program-order execution of a random op chain with the oracle's point
    operations.  Each dataset is padded by chain['halo'] on every side."""
    import ctypes
    import numpy as np
    import oracle
    L = oracle.lib()
    ndim = chain["ndim"]
    h = chain["halo"]
    arrs = [np.array(a, copy=True) for a in data]

    grid = oracle.Grid(ndim, 0, h)
    for lp in chain["loops"]:
        lo, hi = lp["start"], lp["end"]
        if any(b <= a for a, b in zip(lo, hi)):
            continue
        args = lp["args"]
        if lp["op"] == "WSUM":
            oracle.wsum(grid, lo, hi, arrs[args[0]["dat"]], [arrs[a["dat"]] for a in args[1:]],
                        [a["stencil"] for a in args[1:]], lp["params"])
        else:
            l3, h3 = grid.box(lo, hi)
            L.orc_axpby(l3, h3, grid.view(arrs[args[0]["dat"]]), grid.view(arrs[args[1]["dat"]]),
                        ctypes.c_double(lp["params"][0]), ctypes.c_double(lp["params"][1]))
    return arrs


def record_op_chain(ctx, chain, data=None):
    """Declare the chain's datasets / stencils on a context and record its loops."""
    ndim, h = chain["ndim"], chain["halo"]
    blk = ctx.tc_decl_block(ndim)
    dats = [ctx.tc_decl_dat(blk, chain["n"], [h] * ndim, [h] * ndim, None if data is None else data[d])
            for d in range(chain["ndat"])]
    cache = {}

    def st(pts):
        key = tuple(tuple(p) for p in pts)
        if key not in cache:
            cache[key] = ctx.tc_decl_stencil(list(key))
        return cache[key]

    for i, lp in enumerate(chain["loops"]):
        rng = [v for d in range(ndim) for v in (lp["start"][d], lp["end"][d])]
        args = [(dats[a["dat"]], st(a["stencil"]), a["access"]) for a in lp["args"]]
        ctx.tc_par_loop(lp["op"], blk, rng, args, lp["params"], name=f"l{i}")
    return blk, dats
