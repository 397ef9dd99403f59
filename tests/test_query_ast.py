"""Host logic: flattening a WHERE syntax tree (the node shapes of the
Section 4.3 B example) into the expression node list, checked against node
lists written by hand and, through the oracle's plaintext evaluation, against
the query's meaning."""
import itertools

import pytest

from oracle import circuits as C
from paper_2510_15413_amd.query import where_nodes

AGE_SALARY = {
    "type": "SelectStatement", "columns": ["*"], "from": {"type": "Table", "name": "people"},
    "where": {
        "type": "BinaryExpression", "operator": "AND",
        "left": {"type": "ComparisonExpression", "operator": ">",
                 "left": {"type": "Identifier", "name": "age"}, "right": {"type": "Number", "value": 18}},
        "right": {"type": "ComparisonExpression", "operator": "<",
                  "left": {"type": "Identifier", "name": "salary"}, "right": {"type": "Number", "value": 1000}},
    },
}


def test_age_salary_encrypted_literals():
    nodes, lits = where_nodes(AGE_SALARY, {"age": 0, "salary": 1})
    assert lits == [18, 1000]
    assert nodes == [
        {"kind": "column", "col": 0}, {"kind": "literal", "lit": 0}, {"kind": "cmp", "op": "gt", "a": 0, "b": 1},
        {"kind": "column", "col": 1}, {"kind": "literal", "lit": 1}, {"kind": "cmp", "op": "lt", "a": 3, "b": 4},
        {"kind": "and", "a": 2, "b": 5},
    ]


def test_age_salary_plain_matches_semantics():
    nodes, lits = where_nodes(AGE_SALARY, {"age": 0, "salary": 1}, literals="plain")
    assert lits == []
    for age, sal in itertools.product((0, 18, 19, 90), (0, 999, 1000, 2047)):
        assert C.expr_plain(nodes, [age, sal], [], 11) == (age > 18 and sal < 1000)


def test_not_or_and_calls():
    ast = {"type": "UnaryExpression", "operator": "NOT", "argument": {
        "type": "BinaryExpression", "operator": "OR",
        "left": {"type": "ComparisonExpression", "operator": "<=",
                 "left": {"type": "CallExpression", "callee": "max",
                          "arguments": [{"type": "Identifier", "name": "a"}, {"type": "Identifier", "name": "b"}]},
                 "right": {"type": "Number", "value": 5}},
        "right": {"type": "ComparisonExpression", "operator": "<>",
                  "left": {"type": "Identifier", "name": "a"}, "right": {"type": "Identifier", "name": "b"}}}}
    nodes, lits = where_nodes(ast, {"a": 0, "b": 1}, literals="plain")
    for a, b in itertools.product(range(8), repeat=2):
        assert C.expr_plain(nodes, [a, b], [], 3) == (not (max(a, b) <= 5 or a != b))


@pytest.mark.parametrize("bad", [
    {"type": "Identifier", "name": "age"},                                        # not a condition
    {"type": "ComparisonExpression", "operator": "~", "left": {"type": "Number", "value": 1},
     "right": {"type": "Number", "value": 2}},                                    # unknown operator
    {"type": "BinaryExpression", "operator": "AND", "left": {"type": "Number", "value": 1},
     "right": {"type": "Number", "value": 2}},                                    # AND of values
    {"type": "ComparisonExpression", "operator": "=", "left": {"type": "Identifier", "name": "zip"},
     "right": {"type": "Number", "value": 2}},                                    # unknown column
])
def test_rejects(bad):
    with pytest.raises((ValueError, KeyError)):
        where_nodes(bad, {"age": 0})
