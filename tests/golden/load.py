"""Reader for the closed-form fixtures in this folder (expressions the paper
prints, one named matrix or vector per line, '#' comments)."""
import ast
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def load_expressions(name):
    out = {}
    with open(os.path.join(HERE, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, expr = line.split(":", 1)
            out[key.strip()] = ast.parse(expr.strip(), mode="eval")
    return out


def evaluate(tree, env):
    code = compile(tree, "<golden>", "eval")
    return eval(code, {"__builtins__": {}}, dict(env))
