"""Seeded random BLTLc formulas for tests (Sec. 3.1 grammar): nested, over one
species X, every operator, bounded windows."""


def random_formula(r, depth=0, max_depth=3):
    """Random formula text from the random.Random r."""
    k = r.random()
    if depth >= max_depth or k < 0.25:
        return f"X {r.choice(['<=', '>='])} {r.randint(40, 130)}"
    sub = lambda: random_formula(r, depth + 1, max_depth)   # noqa: E731
    lo = round(r.uniform(0.0, 2.0), 2)
    hi = round(lo + r.uniform(0.1, 4.0), 2)
    if k < 0.35:
        return f"!({sub()})"
    if k < 0.45:
        return f"({sub()}) & ({sub()})"
    if k < 0.55:
        return f"({sub()}) | ({sub()})"
    if k < 0.65:
        return f"X[0,{round(r.uniform(0.05, 0.5), 2)}]({sub()})"
    if k < 0.75:
        return f"F[{lo},{hi}]({sub()})"
    if k < 0.85:
        return f"G[{lo},{hi}]({sub()})"
    return f"({sub()}) U[{lo},{hi}] ({sub()})"
