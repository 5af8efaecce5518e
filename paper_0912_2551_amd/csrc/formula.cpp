// formula.cpp -- BLTLc text -> device monitor program (host side).
//
// Syntax (Sec. 3.1): predicates val op val over species counts; !, &, |;
// X^I, U^I; and the derived F^I p = tt U^I p and G^I p = !F^I !p.
// Precedence: unary > U (right associative) > & > |.
//
// The device evaluates a top-level boolean combination of "atoms", each an
// O(1)-register monitor of one temporal operator applied to state formulas
// (boolean combinations of predicates):
//   p                      decided on the initial state
//   p U[a,b] q, F, G       one status
//   X[a,b] p               decided at the first event
//   p U[0,a] (q U[0,b] r)  status + (left operand held so far, latest start)
// Decided atoms freeze; the combination is evaluated in three-valued logic
// after every state and every time step, so a trajectory stops at the first
// prefix that decides the formula (Sec. 3.2).
//
// Any other formula becomes a trace program: the formula tree itself, which
// the kernel evaluates on the states it records (see trace_value).

#include <hip/hip_runtime.h>

#include <cctype>
#include <climits>
#include <cstdint>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "smc_device.h"
#include "smc_internal.h"

namespace smc {

namespace {

struct Expr {
    enum Kind { VAR, CONST, ADD, SUB, MUL, DIV, NEG, SQRT, POW } kind;
    int var = -1;
    double c = 0.0;
    std::unique_ptr<Expr> a, b;
};

struct Node {
    enum Kind { TT, FF, PRED, NOT, AND, OR, NEXT, UNTIL, FIN, GLOB } kind;
    std::unique_ptr<Expr> lhs, rhs;
    int cmp = 0;
    double lo = 0.0, hi = INFINITY;
    std::unique_ptr<Node> a, b;
};

struct Tok {
    enum Kind { NUM, NAME, OP, END } kind;
    std::string s;
};

class Lexer {
  public:
    explicit Lexer(const std::string &text)
    {
        size_t i = 0;
        const size_t n = text.size();
        while (i < n) {
            const char ch = text[i];
            if (std::isspace((unsigned char)ch)) {
                ++i;
                continue;
            }
            if (std::isdigit((unsigned char)ch) || (ch == '.' && i + 1 < n && std::isdigit((unsigned char)text[i + 1]))) {
                size_t j = i;
                while (j < n && (std::isdigit((unsigned char)text[j]) || text[j] == '.')) ++j;
                if (j < n && (text[j] == 'e' || text[j] == 'E')) {
                    size_t k = j + 1;
                    if (k < n && (text[k] == '+' || text[k] == '-')) ++k;
                    if (k < n && std::isdigit((unsigned char)text[k])) {
                        j = k;
                        while (j < n && std::isdigit((unsigned char)text[j])) ++j;
                    }
                }
                toks.push_back({Tok::NUM, text.substr(i, j - i)});
                i = j;
                continue;
            }
            if (std::isalpha((unsigned char)ch) || ch == '_') {
                size_t j = i;
                while (j < n && (std::isalnum((unsigned char)text[j]) || text[j] == '_')) ++j;
                toks.push_back({Tok::NAME, text.substr(i, j - i)});
                i = j;
                continue;
            }
            static const char *two[] = {"<=", ">=", "!=", "==", "&&", "||"};
            bool matched = false;
            for (const char *t : two) {
                if (text.compare(i, 2, t) == 0) {
                    std::string s(t);
                    if (s == "&&") s = "&";
                    if (s == "||") s = "|";
                    toks.push_back({Tok::OP, s});
                    i += 2;
                    matched = true;
                    break;
                }
            }
            if (matched) continue;
            if (std::strchr("+-*/()<>=!&|[],", ch)) {
                toks.push_back({Tok::OP, std::string(1, ch)});
                ++i;
                continue;
            }
            throw ParseFailure(std::string("unexpected character '") + ch + "'");
        }
        toks.push_back({Tok::END, ""});
    }
    std::vector<Tok> toks;
};

class Parser {
  public:
    Parser(const std::string &text, const std::vector<std::string> &names) : lex_(text)
    {
        for (size_t k = 0; k < names.size(); ++k) names_[names[k]] = (int)k;
    }

    std::unique_ptr<Node> parse()
    {
        auto n = disj();
        if (peek().kind != Tok::END) throw ParseFailure("trailing input at '" + peek().s + "'");
        return n;
    }

  private:
    const Tok &peek(size_t k = 0) const
    {
        const size_t j = pos_ + k;
        return j < lex_.toks.size() ? lex_.toks[j] : lex_.toks.back();
    }
    bool is_op(const char *s, size_t k = 0) const { return peek(k).kind == Tok::OP && peek(k).s == s; }
    Tok take() { return lex_.toks[pos_ < lex_.toks.size() - 1 ? pos_++ : pos_]; }
    void expect(const char *s)
    {
        if (!is_op(s)) throw ParseFailure(std::string("expected '") + s + "' near '" + peek().s + "'");
        ++pos_;
    }

    std::unique_ptr<Node> mk(Node::Kind k)
    {
        auto n = std::make_unique<Node>();
        n->kind = k;
        return n;
    }

    std::unique_ptr<Node> disj()
    {
        auto l = conj();
        while (is_op("|")) {
            ++pos_;
            auto n = mk(Node::OR);
            n->a = std::move(l);
            n->b = conj();
            l = std::move(n);
        }
        return l;
    }
    std::unique_ptr<Node> conj()
    {
        auto l = until();
        while (is_op("&")) {
            ++pos_;
            auto n = mk(Node::AND);
            n->a = std::move(l);
            n->b = until();
            l = std::move(n);
        }
        return l;
    }
    std::unique_ptr<Node> until()
    {
        auto l = unary();
        if (peek().kind == Tok::NAME && peek().s == "U") {
            ++pos_;
            auto n = mk(Node::UNTIL);
            interval(n->lo, n->hi);
            n->a = std::move(l);
            n->b = until();
            return n;
        }
        return l;
    }
    double number()
    {
        const Tok t = take();
        if (t.kind == Tok::NAME && (t.s == "inf" || t.s == "Inf" || t.s == "INF")) return INFINITY;
        if (t.kind != Tok::NUM) throw ParseFailure("expected a number near '" + t.s + "'");
        return std::strtod(t.s.c_str(), nullptr);
    }
    void interval(double &lo, double &hi)
    {
        if (is_op("[")) {
            ++pos_;
            lo = number();
            expect(",");
            hi = number();
            expect("]");
        } else if (is_op("<=")) {
            ++pos_;
            lo = 0.0;
            hi = number();
        } else {
            lo = 0.0;
            hi = INFINITY;
        }
        if (!(lo >= 0.0 && lo <= hi)) throw ParseFailure("bad time interval");
    }
    std::unique_ptr<Node> unary()
    {
        const Tok &t = peek();
        if (t.kind == Tok::OP && t.s == "!") {
            ++pos_;
            auto n = mk(Node::NOT);
            n->a = unary();
            return n;
        }
        if (t.kind == Tok::NAME && (t.s == "F" || t.s == "G" || t.s == "X") &&
            (names_.count(t.s) == 0 || is_op("[", 1))) {
            const std::string op = t.s;
            ++pos_;
            auto n = mk(op == "F" ? Node::FIN : op == "G" ? Node::GLOB : Node::NEXT);
            interval(n->lo, n->hi);
            n->a = unary();
            return n;
        }
        if (t.kind == Tok::NAME && (t.s == "true" || t.s == "tt")) {
            ++pos_;
            return mk(Node::TT);
        }
        if (t.kind == Tok::NAME && (t.s == "false" || t.s == "ff")) {
            ++pos_;
            return mk(Node::FF);
        }
        if (is_op("(")) {
            const size_t save = pos_;
            try {
                return predicate();
            } catch (const ParseFailure &) {
                pos_ = save;
            }
            ++pos_;
            auto inner = disj();
            expect(")");
            return inner;
        }
        return predicate();
    }
    std::unique_ptr<Node> predicate()
    {
        auto n = mk(Node::PRED);
        n->lhs = sum();
        const Tok t = take();
        static const char *ops[] = {"<", "<=", ">=", ">", "=", "!="};
        int cmp = -1;
        for (int k = 0; k < 6; ++k)
            if (t.kind == Tok::OP && t.s == ops[k]) cmp = k;
        if (t.kind == Tok::OP && t.s == "==") cmp = CMP_EQ;
        if (cmp < 0) throw ParseFailure("expected a comparison near '" + t.s + "'");
        n->cmp = cmp;
        n->rhs = sum();
        return n;
    }
    std::unique_ptr<Expr> ebin(Expr::Kind k, std::unique_ptr<Expr> a, std::unique_ptr<Expr> b)
    {
        auto e = std::make_unique<Expr>();
        e->kind = k;
        e->a = std::move(a);
        e->b = std::move(b);
        return e;
    }
    std::unique_ptr<Expr> sum()
    {
        auto l = product();
        while (is_op("+") || is_op("-")) {
            const bool add = is_op("+");
            ++pos_;
            l = ebin(add ? Expr::ADD : Expr::SUB, std::move(l), product());
        }
        return l;
    }
    std::unique_ptr<Expr> product()
    {
        auto l = atom();
        while (is_op("*") || is_op("/")) {
            const bool mul = is_op("*");
            ++pos_;
            l = ebin(mul ? Expr::MUL : Expr::DIV, std::move(l), atom());
        }
        return l;
    }
    std::unique_ptr<Expr> atom()
    {
        const Tok t = take();
        auto e = std::make_unique<Expr>();
        if (t.kind == Tok::NUM) {
            e->kind = Expr::CONST;
            e->c = std::strtod(t.s.c_str(), nullptr);
            return e;
        }
        if (t.kind == Tok::OP && t.s == "-") {
            e->kind = Expr::NEG;
            e->a = atom();
            return e;
        }
        if (t.kind == Tok::OP && t.s == "(") {
            auto inner = sum();
            expect(")");
            return inner;
        }
        if (t.kind == Tok::NAME) {
            std::string low = t.s;
            for (auto &ch : low) ch = (char)std::tolower((unsigned char)ch);
            if ((low == "sqrt" || low == "pow") && is_op("(")) {
                ++pos_;
                e->kind = low == "sqrt" ? Expr::SQRT : Expr::POW;
                e->a = sum();
                if (e->kind == Expr::POW) {
                    expect(",");
                    e->b = sum();
                }
                expect(")");
                return e;
            }
            auto it = names_.find(t.s);
            if (it == names_.end()) throw ParseFailure("unknown species '" + t.s + "'");
            e->kind = Expr::VAR;
            e->var = it->second;
            return e;
        }
        throw ParseFailure("unexpected '" + t.s + "'");
    }

    Lexer lex_;
    size_t pos_ = 0;
    std::map<std::string, int> names_;
};

// ---------------------------------------------------------------------------
// Compilation to the device program.
// ---------------------------------------------------------------------------
bool is_state_formula(const Node *n)
{
    switch (n->kind) {
    case Node::TT:
    case Node::FF:
    case Node::PRED: return true;
    case Node::NOT: return is_state_formula(n->a.get());
    case Node::AND:
    case Node::OR: return is_state_formula(n->a.get()) && is_state_formula(n->b.get());
    default: return false;
    }
}

double horizon_of(const Node *n)
{
    switch (n->kind) {
    case Node::TT:
    case Node::FF:
    case Node::PRED: return 0.0;
    case Node::NOT: return horizon_of(n->a.get());
    case Node::AND:
    case Node::OR: return std::fmax(horizon_of(n->a.get()), horizon_of(n->b.get()));
    case Node::NEXT:
    case Node::FIN:
    case Node::GLOB: return n->hi + horizon_of(n->a.get());
    default: return n->hi + std::fmax(horizon_of(n->a.get()), horizon_of(n->b.get()));
    }
}

// Exact linear form sum w_s x_s + c with integer coefficients, if any.
bool linear_form(const Expr *e, std::map<int, double> &w, double &c, double scale)
{
    switch (e->kind) {
    case Expr::VAR: w[e->var] += scale; return true;
    case Expr::CONST: c += scale * e->c; return true;
    case Expr::NEG: return linear_form(e->a.get(), w, c, -scale);
    case Expr::ADD: return linear_form(e->a.get(), w, c, scale) && linear_form(e->b.get(), w, c, scale);
    case Expr::SUB: return linear_form(e->a.get(), w, c, scale) && linear_form(e->b.get(), w, c, -scale);
    case Expr::MUL:
        if (e->a->kind == Expr::CONST) return linear_form(e->b.get(), w, c, scale * e->a->c);
        if (e->b->kind == Expr::CONST) return linear_form(e->a.get(), w, c, scale * e->b->c);
        return false;
    default: return false;
    }
}

bool is_small_int(double v, double lim) { return std::fabs(v) <= lim && std::floor(v) == v; }

// Does every evaluation of this expression stay an integer exactly
// representable in a double?  (Then any evaluation order gives the same value.)
bool integer_exact(const Expr *e)
{
    switch (e->kind) {
    case Expr::VAR: return true;
    case Expr::CONST: return is_small_int(e->c, 1048576.0);
    case Expr::NEG: return integer_exact(e->a.get());
    case Expr::ADD:
    case Expr::SUB: return integer_exact(e->a.get()) && integer_exact(e->b.get());
    case Expr::MUL:
        return (e->a->kind == Expr::CONST && is_small_int(e->a->c, 1048576.0) && integer_exact(e->b.get())) ||
               (e->b->kind == Expr::CONST && is_small_int(e->b->c, 1048576.0) && integer_exact(e->a.get()));
    default: return false;
    }
}

class Compiler {
  public:
    explicit Compiler(MonProg &p) : p_(p) { std::memset(&p_, 0, sizeof(MonProg)); }

    // A formula outside the compact monitor classes: the formula tree itself
    // (a trace program), evaluated by the kernel on the states it records.
    void compile_trace(const Node *root)
    {
        trace_node(root);
        p_.trace = 1;
        p_.horizon = horizon_of(root);
        p_.all_var = 1;
        for (int q = 0; q < p_.n_preds; ++q) p_.all_var &= p_.preds[q].kind == PK_VAR;
    }

    void compile(const Node *root)
    {
        const int top = top_expr(root);
        const int n = p_.n_atoms;
        for (uint32_t tm = 0; tm < (1u << n); ++tm)
            for (uint32_t fm = 0; fm < (1u << n); ++fm) {
                if (tm & fm) continue;
                const int v = eval_top(top, tm, fm);
                const uint32_t idx = tm | (fm << n);
                if (v == 1) p_.topT[idx >> 6] |= 1ull << (idx & 63);
                if (v == 2) p_.topF[idx >> 6] |= 1ull << (idx & 63);
            }
        p_.horizon = horizon_of(root);
        p_.all_var = 1;
        for (int q = 0; q < p_.n_preds; ++q) p_.all_var &= p_.preds[q].kind == PK_VAR;
    }

  private:
    // ---- trace programs ---------------------------------------------------
    int trace_push(int kind, int pred, int a, int b, double lo, double hi)
    {
        if (p_.tr_n >= kMaxTrace) throw Unsupported("formula too large for the GPU trace monitor (32 nodes)");
        TraceNode &N = p_.tnodes[p_.tr_n];
        N.kind = kind;
        N.pred = pred;
        N.a = a;
        N.b = b;
        N.lo = lo;
        N.hi = hi;
        return p_.tr_n++;
    }

    // children first; F I p = tt U I p, G I p = not(tt U I not p) (Sec. 3.1)
    int trace_node(const Node *n)
    {
        switch (n->kind) {
        case Node::TT: return trace_push(TN_TT, -1, -1, -1, 0.0, 0.0);
        case Node::FF: return trace_push(TN_FF, -1, -1, -1, 0.0, 0.0);
        case Node::PRED: return trace_push(TN_PRED, predicate(n), -1, -1, 0.0, 0.0);
        case Node::NOT: {
            const int a = trace_node(n->a.get());
            return trace_push(TN_NOT, -1, a, -1, 0.0, 0.0);
        }
        case Node::AND:
        case Node::OR: {
            const int a = trace_node(n->a.get());
            const int b = trace_node(n->b.get());
            return trace_push(n->kind == Node::AND ? TN_AND : TN_OR, -1, a, b, 0.0, 0.0);
        }
        case Node::NEXT: {
            const int a = trace_node(n->a.get());
            return trace_push(TN_NEXT, -1, a, -1, n->lo, n->hi);
        }
        case Node::FIN: {
            const int tt = trace_push(TN_TT, -1, -1, -1, 0.0, 0.0);
            const int b = trace_node(n->a.get());
            return trace_push(TN_UNTIL, p_.tr_nskip++, tt, b, n->lo, n->hi);
        }
        case Node::GLOB: {
            const int tt = trace_push(TN_TT, -1, -1, -1, 0.0, 0.0);
            const int c = trace_node(n->a.get());
            const int nc = trace_push(TN_NOT, -1, c, -1, 0.0, 0.0);
            const int u = trace_push(TN_UNTIL, p_.tr_nskip++, tt, nc, n->lo, n->hi);
            return trace_push(TN_NOT, -1, u, -1, 0.0, 0.0);
        }
        default: {
            const int a = trace_node(n->a.get());
            const int b = trace_node(n->b.get());
            return trace_push(TN_UNTIL, p_.tr_nskip++, a, b, n->lo, n->hi);
        }
        }
    }

    // ---- top level: boolean combination of monitors ---------------------
    struct TNode {
        int kind;   // 0 atom, 1 not, 2 and, 3 or
        int a, b, atom;
    };

    int push_top(int kind, int a, int b, int atom)
    {
        tops_.push_back({kind, a, b, atom});
        return (int)tops_.size() - 1;
    }

    // Kleene value of the combination: 0 open, 1 true, 2 false.
    int eval_top(int i, uint32_t tm, uint32_t fm) const
    {
        const TNode &t = tops_[i];
        if (t.kind == 0) return ((tm >> t.atom) & 1u) ? 1 : (((fm >> t.atom) & 1u) ? 2 : 0);
        if (t.kind == 1) {
            const int v = eval_top(t.a, tm, fm);
            return v == 0 ? 0 : 3 - v;
        }
        const int x = eval_top(t.a, tm, fm), y = eval_top(t.b, tm, fm);
        if (t.kind == 2) {
            if (x == 2 || y == 2) return 2;
            return (x == 1 && y == 1) ? 1 : 0;
        }
        if (x == 1 || y == 1) return 1;
        return (x == 2 && y == 2) ? 2 : 0;
    }

    int new_atom()
    {
        if (p_.n_atoms >= kMaxAtoms) throw Unsupported("more than 4 temporal monitors in one formula");
        Atom &a = p_.atoms[p_.n_atoms];
        a.p1 = a.p2 = a.p3 = -1;
        a.slot = -1;
        return p_.n_atoms++;
    }

    int top_expr(const Node *n)
    {
        if (is_state_formula(n)) {
            const int a = new_atom();
            p_.atoms[a].kind = AK_PROP;
            p_.atoms[a].p1 = prop(n, false);
            return push_top(0, -1, -1, a);
        }
        switch (n->kind) {
        case Node::NOT: return push_top(1, top_expr(n->a.get()), -1, -1);
        case Node::AND:
        case Node::OR: {
            const int x = top_expr(n->a.get());
            const int y = top_expr(n->b.get());
            return push_top(n->kind == Node::AND ? 2 : 3, x, y, -1);
        }
        case Node::FIN:
        case Node::GLOB: {
            if (!is_state_formula(n->a.get())) {
                int r = response(n);
                // F I (q U[0,b] r) and F I F[0,b] r: the nested until with p = true
                if (r < 0 && n->kind == Node::FIN) r = nested(nullptr, n);
                if (r >= 0) return push_top(0, -1, -1, r);
                throw Unsupported("F/G over a temporal formula is outside the GPU monitor classes");
            }
            const int a = new_atom();
            Atom &A = p_.atoms[a];
            A.kind = AK_UNTIL;
            A.neg = n->kind == Node::GLOB;
            A.lo = n->lo;
            A.hi = n->hi;
            A.p1 = prop_true();
            A.p2 = prop(n->a.get(), n->kind == Node::GLOB);
            return push_top(0, -1, -1, a);
        }
        case Node::NEXT: {
            if (!is_state_formula(n->a.get())) {
                const int r = next_until(n);
                if (r >= 0) return push_top(0, -1, -1, r);
                throw Unsupported("X over a temporal formula is outside the GPU monitor classes");
            }
            const int a = new_atom();
            Atom &A = p_.atoms[a];
            A.kind = AK_NEXT;
            A.lo = n->lo;
            A.hi = n->hi;
            A.p1 = prop(n->a.get(), false);
            return push_top(0, -1, -1, a);
        }
        case Node::UNTIL: {
            const Node *l = n->a.get(), *r = n->b.get();
            if (!is_state_formula(l))
                throw Unsupported("the left operand of U must be a state formula on the GPU");
            if (is_state_formula(r)) {
                const int a = new_atom();
                Atom &A = p_.atoms[a];
                A.kind = AK_UNTIL;
                A.lo = n->lo;
                A.hi = n->hi;
                A.p1 = prop(l, false);
                A.p2 = prop(r, false);
                return push_top(0, -1, -1, a);
            }
            int a = nested(l, n);
            if (a < 0) a = until_glob(l, n);
            if (a < 0)
                throw Unsupported("nested until needs the form p U[a,b] (q U[0,c] r) or p U[a,b] (r & G[0,c] q)");
            return push_top(0, -1, -1, a);
        }
        default: throw Unsupported("formula outside the GPU monitor classes");
        }
    }

    // p U[a,b] (q U[0,c] r) or p U[a,b] F[0,c] r, where n is the outer until
    // (or the outer F, with l = nullptr standing for p = true).  Returns the
    // monitor, or -1 when the inner formula has neither form.
    int nested(const Node *l, const Node *n)
    {
        const Node *r = l ? n->b.get() : n->a.get();
        const bool inner_until = r->kind == Node::UNTIL && is_state_formula(r->a.get()) &&
                                 is_state_formula(r->b.get());
        const bool inner_fin = r->kind == Node::FIN && is_state_formula(r->a.get());
        if (!(inner_until || inner_fin) || r->lo != 0.0) return -1;
        const int slot = time_slot();
        const int a = new_atom();
        Atom &A = p_.atoms[a];
        A.kind = AK_NESTED;
        A.slot = slot;
        A.lo = n->lo;
        A.hi = n->hi;
        A.hi2 = r->hi;
        A.p1 = l ? prop(l, false) : prop_true();
        if (inner_until) {
            A.p2 = prop(r->a.get(), false);
            A.p3 = prop(r->b.get(), false);
        } else {
            A.p2 = prop_true();
            A.p3 = prop(r->a.get(), false);
        }
        return a;
    }

    // p U[a,b] (r & G[0,c] q), either conjunct order, r optional, where n is
    // the until and l its left operand; -1 for any other right operand.
    int until_glob(const Node *l, const Node *n)
    {
        const Node *r = n->b.get();
        auto is_g = [&](const Node *m) {
            return m->kind == Node::GLOB && m->lo == 0.0 && is_state_formula(m->a.get());
        };
        const Node *g = nullptr, *side = nullptr;
        if (is_g(r)) {
            g = r;
        } else if (r->kind == Node::AND) {
            const Node *x = r->a.get(), *y = r->b.get();
            if (is_state_formula(x) && is_g(y)) side = x, g = y;
            else if (is_state_formula(y) && is_g(x)) side = y, g = x;
        }
        if (!g) return -1;
        const int slot = time_slot();
        const int a = new_atom();
        Atom &A = p_.atoms[a];
        A.kind = AK_UNTILG;
        A.slot = slot;
        A.lo = n->lo;
        A.hi = n->hi;
        A.hi2 = g->hi;
        A.p1 = prop(l, false);
        A.p2 = prop(g->a.get(), false);
        A.p3 = side ? prop(side, false) : prop_true();
        return a;
    }

    // X I (p U J q), X I F J q and X I G J q, where n is the X node; -1 for
    // any other operand.
    int next_until(const Node *n)
    {
        const Node *u = n->a.get();
        const bool until = u->kind == Node::UNTIL && is_state_formula(u->a.get()) &&
                           is_state_formula(u->b.get());
        const bool fin_glob = (u->kind == Node::FIN || u->kind == Node::GLOB) && is_state_formula(u->a.get());
        if (!until && !fin_glob) return -1;
        const int slot = time_slot();
        const int a = new_atom();
        Atom &A = p_.atoms[a];
        A.kind = AK_NEXTU;
        A.slot = slot;
        A.lo = n->lo;
        A.hi = n->hi;
        A.lo2 = u->lo;
        A.hi2 = u->hi;
        A.neg = u->kind == Node::GLOB ? 1 : 0;
        if (until) {
            A.p1 = prop(u->a.get(), false);
            A.p2 = prop(u->b.get(), false);
        } else {
            A.p1 = prop_true();
            A.p2 = prop(u->a.get(), u->kind == Node::GLOB);
        }
        return a;
    }

    // A free per-lane time register for a nested, response, next-until or
    // until-G monitor.
    int time_slot() const
    {
        int slot = 0;
        for (int k = 0; k < p_.n_atoms; ++k)
            if (p_.atoms[k].kind == AK_NESTED || p_.atoms[k].kind == AK_RESP || p_.atoms[k].kind == AK_NEXTU ||
                p_.atoms[k].kind == AK_UNTILG)
                ++slot;
        if (slot >= kMaxNested) throw Unsupported("more than two monitors with a time register");
        return slot;
    }

    // G[lo,hi](s1 | F[0,d] s2), with either operand order and s1 optional, or
    // its dual F[lo,hi](a & G[0,d] b) = !G[lo,hi](!a | F[0,d] !b).  Returns the
    // monitor, or -1 when the formula has neither form.
    int response(const Node *n)
    {
        const bool glob = n->kind == Node::GLOB;
        const Node *body = n->a.get();
        const Node::Kind inner = glob ? Node::FIN : Node::GLOB;
        const Node::Kind join = glob ? Node::OR : Node::AND;
        auto is_inner = [&](const Node *m) {
            return m->kind == inner && m->lo == 0.0 && is_state_formula(m->a.get());
        };
        const Node *side = nullptr, *tmp = nullptr;
        if (is_inner(body)) {
            tmp = body;
        } else if (body->kind == join) {
            const Node *x = body->a.get(), *y = body->b.get();
            if (is_state_formula(x) && is_inner(y)) side = x, tmp = y;
            else if (is_state_formula(y) && is_inner(x)) side = y, tmp = x;
        }
        if (!tmp) return -1;
        const int slot = time_slot();
        const int a = new_atom();
        Atom &A = p_.atoms[a];
        A.kind = AK_RESP;
        A.neg = glob ? 0 : 1;
        A.slot = slot;
        A.lo = n->lo;
        A.hi = n->hi;
        A.hi2 = tmp->hi;
        // the G form's operands as they are, the F form's negated; a missing
        // side is s1 = false (G form) or a = true (F form), false either way
        A.p1 = side ? prop(side, !glob) : prop_const(false);
        A.p2 = prop(tmp->a.get(), !glob);
        return a;
    }

    // ---- state formulas: truth tables over contiguous predicates ----------
    struct PNode {
        int kind;   // 0 tt, 1 ff, 2 pred, 3 not, 4 and, 5 or
        int a, b, local;
    };

    int build_prop(const Node *n, std::vector<PNode> &tree, int off)
    {
        PNode q{0, -1, -1, -1};
        switch (n->kind) {
        case Node::TT: q.kind = 0; break;
        case Node::FF: q.kind = 1; break;
        case Node::PRED:
            q.kind = 2;
            q.local = predicate(n) - off;
            break;
        case Node::NOT:
            q.kind = 3;
            q.a = build_prop(n->a.get(), tree, off);
            break;
        default:
            q.kind = n->kind == Node::AND ? 4 : 5;
            q.a = build_prop(n->a.get(), tree, off);
            q.b = build_prop(n->b.get(), tree, off);
            break;
        }
        tree.push_back(q);
        return (int)tree.size() - 1;
    }

    static bool eval_prop(const std::vector<PNode> &tree, int i, uint32_t bits)
    {
        const PNode &q = tree[i];
        switch (q.kind) {
        case 0: return true;
        case 1: return false;
        case 2: return (bits >> q.local) & 1u;
        case 3: return !eval_prop(tree, q.a, bits);
        case 4: return eval_prop(tree, q.a, bits) && eval_prop(tree, q.b, bits);
        default: return eval_prop(tree, q.a, bits) || eval_prop(tree, q.b, bits);
        }
    }

    int finish_prop(int off, int cnt, uint32_t table)
    {
        if (p_.n_props >= kMaxProps) throw Unsupported("too many state formulas");
        Prop &P = p_.props[p_.n_props];
        P.off = off;
        P.cnt = cnt;
        P.table = table;
        return p_.n_props++;
    }

    int prop_true() { return finish_prop(0, 0, 1u); }
    int prop_const(bool v) { return finish_prop(0, 0, v ? 1u : 0u); }

    int prop(const Node *n, bool negate)
    {
        const int off = p_.n_preds;
        std::vector<PNode> tree;
        const int root = build_prop(n, tree, off);
        const int cnt = p_.n_preds - off;
        if (cnt > kMaxPropPreds) throw Unsupported("a state formula uses more than 5 predicates");
        uint32_t table = 0;
        for (uint32_t bits = 0; bits < (1u << cnt); ++bits)
            if (eval_prop(tree, root, bits) != negate) table |= 1u << bits;
        return finish_prop(off, cnt, table);
    }

    // ---- predicates -------------------------------------------------------
    static int mirror(int op)
    {
        switch (op) {
        case CMP_LT: return CMP_GT;
        case CMP_LE: return CMP_GE;
        case CMP_GE: return CMP_LE;
        case CMP_GT: return CMP_LT;
        default: return op;
        }
    }

    int predicate(const Node *n)
    {
        if (p_.n_preds >= kMaxPreds) throw Unsupported("more than 16 predicates");
        const int id = p_.n_preds++;
        Pred &P = p_.preds[id];
        P.op = n->cmp;
        const Expr *l = n->lhs.get(), *r = n->rhs.get();
        auto int32_const = [](const Expr *e) {
            return e->kind == Expr::CONST && std::floor(e->c) == e->c && std::fabs(e->c) <= 2147483647.0;
        };
        if ((l->kind == Expr::VAR && int32_const(r)) || (r->kind == Expr::VAR && int32_const(l))) {
            const bool left = l->kind == Expr::VAR;
            P.kind = PK_VAR;
            P.var = left ? l->var : r->var;
            P.c32 = (int32_t)(left ? r->c : l->c);
            P.op = left ? n->cmp : mirror(n->cmp);
            // x op c as a range test lo <= x <= hi, possibly negated
            const int32_t c = P.c32, mn = INT32_MIN, mx = INT32_MAX;
            switch (P.op) {
            case CMP_GE: P.lo32 = c; P.hi32 = mx; P.neg = 0; break;
            case CMP_LT: P.lo32 = c; P.hi32 = mx; P.neg = 1; break;
            case CMP_LE: P.lo32 = mn; P.hi32 = c; P.neg = 0; break;
            case CMP_GT: P.lo32 = mn; P.hi32 = c; P.neg = 1; break;
            case CMP_EQ: P.lo32 = c; P.hi32 = c; P.neg = 0; break;
            default: P.lo32 = c; P.hi32 = c; P.neg = 1; break;
            }
            return id;
        }
        std::map<int, double> w;
        double c = 0.0;
        const bool lin = integer_exact(l) && integer_exact(r) && linear_form(l, w, c, 1.0) &&
                         linear_form(r, w, c, -1.0);
        std::vector<std::pair<int, double>> terms;
        for (auto &kv : w)
            if (kv.second != 0.0) terms.push_back(kv);
        bool ok = lin && terms.size() <= 4 && is_small_int(c, 1125899906842624.0);
        for (auto &tm : terms) ok = ok && is_small_int(tm.second, 1048576.0);
        if (ok) {
            P.kind = PK_LINEAR;
            P.nterm = (int)terms.size();
            for (int k = 0; k < P.nterm; ++k) {
                P.vars[k] = terms[k].first;
                P.w[k] = (int64_t)terms[k].second;
            }
            P.c = (int64_t)c;
            return id;
        }
        P.kind = PK_RPN;
        P.lhs_off = n_vops_;
        int depth = 0, maxd = 0;
        val(l, depth, maxd);
        P.lhs_len = n_vops_ - P.lhs_off;
        P.rhs_off = n_vops_;
        depth = 0;
        val(r, depth, maxd);
        P.rhs_len = n_vops_ - P.rhs_off;
        if (maxd > kValStack) throw Unsupported("arithmetic predicate too deep for the GPU");
        return id;
    }

    void emit_val(int op, int var, double c, int &depth, int &maxd, int delta)
    {
        if (n_vops_ >= kMaxValOps) throw Unsupported("arithmetic predicates too long");
        p_.vop[n_vops_] = op;
        p_.vvar[n_vops_] = var;
        p_.vconst[n_vops_] = c;
        ++n_vops_;
        depth += delta;
        if (depth > maxd) maxd = depth;
    }

    void val(const Expr *e, int &depth, int &maxd)
    {
        switch (e->kind) {
        case Expr::VAR: emit_val(VO_VAR, e->var, 0.0, depth, maxd, +1); return;
        case Expr::CONST: emit_val(VO_CONST, 0, e->c, depth, maxd, +1); return;
        case Expr::NEG:
            val(e->a.get(), depth, maxd);
            emit_val(VO_NEG, 0, 0.0, depth, maxd, 0);
            return;
        case Expr::SQRT:
            val(e->a.get(), depth, maxd);
            emit_val(VO_SQRT, 0, 0.0, depth, maxd, 0);
            return;
        case Expr::POW: {
            // pow(v, k) with a constant integral k in 0..64: binary powering
            // (see powi in the kernels); other exponents have no
            // bit-reproducible form here
            const Expr *k = e->b.get();
            if (k->kind != Expr::CONST || !(k->c >= 0.0 && k->c <= 64.0) || k->c != std::floor(k->c))
                throw Unsupported("pow() on the GPU takes a constant integral exponent in 0..64");
            val(e->a.get(), depth, maxd);
            emit_val(VO_POWI, (int)k->c, 0.0, depth, maxd, 0);
            return;
        }
        default: {
            val(e->a.get(), depth, maxd);
            val(e->b.get(), depth, maxd);
            const int op = e->kind == Expr::ADD ? VO_ADD : e->kind == Expr::SUB ? VO_SUB
                           : e->kind == Expr::MUL ? VO_MUL : VO_DIV;
            emit_val(op, 0, 0.0, depth, maxd, -1);
            return;
        }
        }
    }

    MonProg &p_;
    std::vector<TNode> tops_;
    int n_vops_ = 0;
};

}  // namespace

void compile_formula(const std::string &text, const std::vector<std::string> &names, MonProg &out)
{
    Parser ps(text, names);
    auto root = ps.parse();
    try {
        Compiler cc(out);
        cc.compile(root.get());
    } catch (const Unsupported &) {
        // outside the compact monitor classes: a trace program (its own
        // limits, e.g. on predicates, still apply)
        Compiler tc(out);
        tc.compile_trace(root.get());
    }
}

}  // namespace smc
