"""From a WHERE clause's syntax tree to the node list of ``sql_expr_eval``.

Section 4.3 B turns the WHERE clause into a homomorphic expression tree whose
leaves are operands (column identifiers, numbers) and whose inner nodes are
operators carried as plaintext metadata; its example is a JSON syntax tree of
BinaryExpression / ComparisonExpression / Identifier / Number nodes.  This
module flattens such a tree (the same node shapes, plus UnaryExpression NOT and
max/min calls) into the topologically ordered node list the library takes.
Numbers become encrypted literals (the client encrypts them, as EncryptQuery
does) or plaintext constants.  Pure host logic: no arithmetic on ciphertexts.
"""
from __future__ import annotations

CMP_OPERATORS = {"=": "eq", "==": "eq", "!=": "ne", "<>": "ne", "<": "lt", "<=": "le", ">": "gt", ">=": "ge"}
BOOL_OPERATORS = {"AND": "and", "OR": "or", "XOR": "xor"}
CALLS = {"max": "max", "min": "min"}


def where_nodes(ast, columns, literals="encrypted"):
    """Flatten a WHERE syntax tree.

    ast: the tree (or a SelectStatement, whose "where" is used).  columns:
    mapping from identifier name to column index.  literals: "encrypted" (each
    Number becomes a literal node; the values to encrypt are returned in
    order) or "plain" (Numbers become plaintext constants).
    Returns (nodes, literal_values)."""
    if literals not in ("encrypted", "plain"):
        raise ValueError("literals must be 'encrypted' or 'plain'")
    if isinstance(ast, dict) and ast.get("type") == "SelectStatement":
        ast = ast.get("where")
    if ast is None:
        raise ValueError("no WHERE clause")
    nodes, lits = [], []

    def emit(nd):
        nodes.append(nd)
        return len(nodes) - 1

    def walk(t):
        kind = t.get("type")
        if kind == "Identifier":
            name = t["name"]
            if name not in columns:
                raise KeyError(f"unknown column {name!r}")
            return emit({"kind": "column", "col": int(columns[name])}), "value"
        if kind == "Number":
            v = int(t["value"])
            if v < 0:
                raise ValueError("negative literal")
            if literals == "plain":
                return emit({"kind": "const", "value": v}), "value"
            lits.append(v)
            return emit({"kind": "literal", "lit": len(lits) - 1}), "value"
        if kind == "ComparisonExpression":
            op = CMP_OPERATORS.get(t["operator"])
            if op is None:
                raise ValueError(f"unsupported comparison {t['operator']!r}")
            a, ka = walk(t["left"])
            b, kb = walk(t["right"])
            if ka != "value" or kb != "value":
                raise ValueError("comparison operands must be values")
            return emit({"kind": "cmp", "op": op, "a": a, "b": b}), "bool"
        if kind == "BinaryExpression":
            op = BOOL_OPERATORS.get(str(t["operator"]).upper())
            if op is None:
                raise ValueError(f"unsupported operator {t['operator']!r}")
            a, ka = walk(t["left"])
            b, kb = walk(t["right"])
            if ka != "bool" or kb != "bool":
                raise ValueError(f"{op} takes conditions")
            return emit({"kind": op, "a": a, "b": b}), "bool"
        if kind == "UnaryExpression":
            if str(t["operator"]).upper() != "NOT":
                raise ValueError(f"unsupported unary operator {t['operator']!r}")
            a, ka = walk(t["argument"])
            if ka != "bool":
                raise ValueError("NOT takes a condition")
            return emit({"kind": "not", "a": a}), "bool"
        if kind == "CallExpression":
            fn = CALLS.get(str(t["callee"]).lower())
            args = t.get("arguments", [])
            if fn is None or len(args) != 2:
                raise ValueError("calls: max(a, b) and min(a, b)")
            a, ka = walk(args[0])
            b, kb = walk(args[1])
            if ka != "value" or kb != "value":
                raise ValueError(f"{fn} takes values")
            return emit({"kind": fn, "a": a, "b": b}), "value"
        raise ValueError(f"unsupported node type {kind!r}")

    _, root_kind = walk(ast)
    if root_kind != "bool":
        raise ValueError("a WHERE clause must be a condition")
    return nodes, lits
