"""Seeded random BLTLc formulas for tests (Sec. 3.1 grammar): nested, every
operator, bounded windows, predicates comparing one species with a constant."""


def random_formula(r, depth=0, max_depth=3, names=("X",), lo=40, hi=130, around=None):
    """Random formula text from the random.Random r; predicates compare a
    species of `names` with a constant in [lo, hi], or in [c + lo, c + hi]
    around the species' value c in the dict `around`."""
    k = r.random()
    if depth >= max_depth or k < 0.25:
        name = r.choice(list(names))
        c = around[name] if around else 0
        return f"{name} {r.choice(['<=', '>='])} {max(0, c + r.randint(lo, hi))}"
    sub = lambda: random_formula(r, depth + 1, max_depth, names, lo, hi, around)   # noqa: E731
    wlo = round(r.uniform(0.0, 2.0), 2)
    whi = round(wlo + r.uniform(0.1, 4.0), 2)
    if k < 0.35:
        return f"!({sub()})"
    if k < 0.45:
        return f"({sub()}) & ({sub()})"
    if k < 0.55:
        return f"({sub()}) | ({sub()})"
    if k < 0.65:
        return f"X[0,{round(r.uniform(0.05, 0.5), 2)}]({sub()})"
    if k < 0.75:
        return f"F[{wlo},{whi}]({sub()})"
    if k < 0.85:
        return f"G[{wlo},{whi}]({sub()})"
    return f"({sub()}) U[{wlo},{whi}] ({sub()})"
