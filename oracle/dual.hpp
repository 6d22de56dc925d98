// Forward-mode dual numbers for the CPU oracle (test infrastructure only).
//
// Dual<N,T> carries a value and N first-order tangents.  Nesting
// (Dual<8, Dual<6>>) gives mixed second derivatives: the oracle uses it to
// differentiate the gradient of the Hamiltonian with respect to the six star
// parameters.  Every derivative the oracle needs (the right-hand side of
// Hamilton's equations, surface gradients, the forward-mode parameter
// tangents) comes from this one generic mechanism instead of hand-derived
// formulas, so the oracle and the GPU path share no derivative code.
#pragma once
#include <cmath>
#include <type_traits>

namespace orc {

template <int N, class T = double>
struct Dual {
    T v;
    T d[N];
    Dual() : v(0) { for (int i = 0; i < N; ++i) d[i] = T(0); }
    Dual(double c) : v(c) { for (int i = 0; i < N; ++i) d[i] = T(0); }
    template <class U, class = std::enable_if_t<std::is_same<U, T>::value && !std::is_same<U, double>::value>>
    Dual(const U& c) : v(c) { for (int i = 0; i < N; ++i) d[i] = T(0); }
    static Dual var(const T& x, int i) { Dual r(x); r.d[i] = T(1); return r; }
};

template <class X> struct is_dual : std::false_type {};
template <int N, class T> struct is_dual<Dual<N, T>> : std::true_type {};

// plain value of any (possibly nested) scalar
inline double val(double x) { return x; }
template <int N, class T> inline double val(const Dual<N, T>& x) { return val(x.v); }

// ---- Dual (op) Dual ----
template <int N, class T> inline Dual<N, T> operator+(const Dual<N, T>& a, const Dual<N, T>& b) {
    Dual<N, T> r; r.v = a.v + b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
    return r; }
template <int N, class T> inline Dual<N, T> operator-(const Dual<N, T>& a, const Dual<N, T>& b) {
    Dual<N, T> r; r.v = a.v - b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
    return r; }
template <int N, class T> inline Dual<N, T> operator*(const Dual<N, T>& a, const Dual<N, T>& b) {
    Dual<N, T> r; r.v = a.v * b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r; }
template <int N, class T> inline Dual<N, T> operator/(const Dual<N, T>& a, const Dual<N, T>& b) {
    Dual<N, T> r; r.v = a.v / b.v;
    for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
    return r; }
template <int N, class T> inline Dual<N, T> operator-(const Dual<N, T>& a) {
    Dual<N, T> r; r.v = -a.v; for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
    return r; }

// ---- Dual (op) scalar, scalar (op) Dual; scalar = double or the inner type T ----
template <int N, class T, class U>
using enable_scalar = std::enable_if_t<!std::is_same<U, Dual<N, T>>::value &&
                                       (std::is_same<U, double>::value || std::is_same<U, T>::value)>;

template <int N, class T, class U, class = enable_scalar<N, T, U>>
inline Dual<N, T> operator+(const Dual<N, T>& a, const U& b) { Dual<N, T> r = a; r.v = a.v + b; return r; }
template <int N, class T, class U, class = enable_scalar<N, T, U>>
inline Dual<N, T> operator+(const U& b, const Dual<N, T>& a) { Dual<N, T> r = a; r.v = b + a.v; return r; }
template <int N, class T, class U, class = enable_scalar<N, T, U>>
inline Dual<N, T> operator-(const Dual<N, T>& a, const U& b) { Dual<N, T> r = a; r.v = a.v - b; return r; }
template <int N, class T, class U, class = enable_scalar<N, T, U>>
inline Dual<N, T> operator-(const U& b, const Dual<N, T>& a) {
    Dual<N, T> r; r.v = b - a.v; for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
    return r; }
template <int N, class T, class U, class = enable_scalar<N, T, U>>
inline Dual<N, T> operator*(const Dual<N, T>& a, const U& b) {
    Dual<N, T> r; r.v = a.v * b; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b;
    return r; }
template <int N, class T, class U, class = enable_scalar<N, T, U>>
inline Dual<N, T> operator*(const U& b, const Dual<N, T>& a) {
    Dual<N, T> r; r.v = b * a.v; for (int i = 0; i < N; ++i) r.d[i] = b * a.d[i];
    return r; }
template <int N, class T, class U, class = enable_scalar<N, T, U>>
inline Dual<N, T> operator/(const Dual<N, T>& a, const U& b) {
    Dual<N, T> r; r.v = a.v / b; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] / b;
    return r; }
template <int N, class T, class U, class = enable_scalar<N, T, U>>
inline Dual<N, T> operator/(const U& b, const Dual<N, T>& a) {
    Dual<N, T> r; r.v = b / a.v;
    for (int i = 0; i < N; ++i) r.d[i] = -(b * a.d[i]) / (a.v * a.v);
    return r; }

template <int N, class T, class U> inline Dual<N, T>& operator+=(Dual<N, T>& a, const U& b) { a = a + b; return a; }
template <int N, class T, class U> inline Dual<N, T>& operator-=(Dual<N, T>& a, const U& b) { a = a - b; return a; }
template <int N, class T, class U> inline Dual<N, T>& operator*=(Dual<N, T>& a, const U& b) { a = a * b; return a; }
template <int N, class T, class U> inline Dual<N, T>& operator/=(Dual<N, T>& a, const U& b) { a = a / b; return a; }

// comparisons act on the plain value
template <class A, class B, class = std::enable_if_t<is_dual<A>::value || is_dual<B>::value>>
inline bool operator<(const A& a, const B& b) { return val(a) < val(b); }
template <class A, class B, class = std::enable_if_t<is_dual<A>::value || is_dual<B>::value>>
inline bool operator>(const A& a, const B& b) { return val(a) > val(b); }
template <class A, class B, class = std::enable_if_t<is_dual<A>::value || is_dual<B>::value>>
inline bool operator<=(const A& a, const B& b) { return val(a) <= val(b); }
template <class A, class B, class = std::enable_if_t<is_dual<A>::value || is_dual<B>::value>>
inline bool operator>=(const A& a, const B& b) { return val(a) >= val(b); }

// ---- elementary functions (chain rule written out) ----
using std::sqrt; using std::sin; using std::cos; using std::exp; using std::log;
using std::fabs; using std::atan2; using std::acos; using std::floor;

template <int N, class T> inline Dual<N, T> sqrt(const Dual<N, T>& a) {
    Dual<N, T> r; r.v = sqrt(a.v); T g = 0.5 / r.v;
    for (int i = 0; i < N; ++i) r.d[i] = g * a.d[i];
    return r; }
template <int N, class T> inline Dual<N, T> sin(const Dual<N, T>& a) {
    Dual<N, T> r; r.v = sin(a.v); T g = cos(a.v);
    for (int i = 0; i < N; ++i) r.d[i] = g * a.d[i];
    return r; }
template <int N, class T> inline Dual<N, T> cos(const Dual<N, T>& a) {
    Dual<N, T> r; r.v = cos(a.v); T g = -sin(a.v);
    for (int i = 0; i < N; ++i) r.d[i] = g * a.d[i];
    return r; }
template <int N, class T> inline Dual<N, T> exp(const Dual<N, T>& a) {
    Dual<N, T> r; r.v = exp(a.v);
    for (int i = 0; i < N; ++i) r.d[i] = r.v * a.d[i];
    return r; }
template <int N, class T> inline Dual<N, T> log(const Dual<N, T>& a) {
    Dual<N, T> r; r.v = log(a.v);
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] / a.v;
    return r; }
// |a|: derivative sign(a); at a == 0 the one-sided derivative of +a is used
template <int N, class T> inline Dual<N, T> fabs(const Dual<N, T>& a) { return (val(a) < 0.0) ? -a : a; }
template <int N, class T> inline Dual<N, T> atan2(const Dual<N, T>& y, const Dual<N, T>& x) {
    Dual<N, T> r; r.v = atan2(y.v, x.v); T den = x.v * x.v + y.v * y.v;
    for (int i = 0; i < N; ++i) r.d[i] = (x.v * y.d[i] - y.v * x.d[i]) / den;
    return r; }
template <int N, class T> inline Dual<N, T> floor(const Dual<N, T>& a) { return Dual<N, T>(floor(a.v)); }

}  // namespace orc
